// gna.hip - HIP (gfx950) implementation of the C ABI declared in include/gna.h.
//
// Kernels:
//   k_prepare        FP64 theta -> MFMA weight fragments, bias, embedding table
//   k_logpsi         log psi of each sample (Eq. 1 + two-head readout)
//   k_eloc           log psi of every bond-exchanged configuration, FP64
//                    compensated sums of psi(s^ij)/psi(s) per (sample, bond chunk)
//   k_eloc_finalize  diagonal and field terms + chunk partials -> E_loc, evaluation count
//   k_sweep          Metropolis spin-swap chains (Philox4x32-10 draws)
//   k_inc_base, k_eloc_inc, k_sweep_inc   receptive-field (incremental) evaluation
//                    of the local energy and the sampler's proposals (gna_inc.h)
//   k_eloc_pipe, k_sweep_pipe   the same with the layers of several jobs pipelined
//                    (gna_pipe.h, instantiated in gna_pipe.hip)
//   k_isgo_stats     ISGO weights, energy, variance, ESS, cotangents (FP64)
//   k_vjp_* / k_vjp_reduce   reverse pass (FP32, FP64 for FP64), deterministic reduction
//   k_sgd            theta -= alpha * grad
//   k_group_*        grouping of duplicated configurations with counts
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "gna.h"
#include "gna_kernels.h"
#include "gna_vjp.h"
#include "gna_inc.h"
#include "gna_pipe.h"
#include "gna_pipe_api.h"

using namespace gna;

// Scratch of gna_local_energy_noalloc (per-call base log psi, per-item partial sums
// and counts, the evaluation counter): a file-scope device array, one copy per GPU,
// held until the process ends.  Host code never passes its name to a kernel: the
// device address of each GPU's copy comes from hipGetSymbolAddress at gna_init.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// ===========================================================================
// Device kernels
// ===========================================================================

// Build the per-precision device weights from FP64 theta.
//   wfrag[w][s][t][lane][j] = W[w][blk*F + kk][row_feature(16t + lane%16)],
//   s < F/KS: message block (blk 0), else self block (blk 1);
//   kk = KS*(s mod F/KS) + VEC*(lane/16) + j.
//   Split weights (P::WBLK = 2): each layer's block is followed by the lo parts.
//   act 0 (tanh): W and b are multiplied by P::kScale, the argument scaling that
//   P::act expects; act 1 (ReLU + layer normalisation): unscaled.  The embedding
//   rows are f(W_e[x] + b_e) in FP64, rounded once.
template <class P, int F>
__global__ void k_prepare(const double* __restrict__ theta, int nW, int act, void* wfrag, void* bias,
                          void* emb) {
  using WT = typename P::WT;
  using Acc = typename P::Acc;
  constexpr int KSB = F / P::KS, MT = F / 16, VEC = P::VEC;
  const double* We = theta;
  const double* be = theta + 2 * F;
  const double* W = theta + 3 * F;
  const double* b = W + (size_t)nW * 2 * F * F;
  WT* wf = reinterpret_cast<WT*>(wfrag);
  const int per_layer = 2 * F * F;
  const int total = nW * per_layer;
  const double scale = act == 0 ? P::kScale : 1.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    int r = e;
    const int j = r % VEC; r /= VEC;
    const int lane = r % 64; r /= 64;
    const int t = r % MT; r /= MT;
    const int s = r % (2 * KSB); r /= (2 * KSB);
    const int w = r;
    const int blk = s / KSB, ss = s % KSB;
    const int kk = P::KS * ss + VEC * (lane / 16) + j;
    const int f = P::row_feature(16 * t + lane % 16);
    const double v = W[(size_t)w * per_layer + (size_t)(blk * F + kk) * F + f];
    if constexpr (P::WBLK == 1) {
      wf[e] = P::to_w(scale * v);
    } else {   // a layer's block: its hi fragments, then its lo fragments
      const size_t hi = (size_t)e + (size_t)w * per_layer;
      wf[hi] = P::to_w(scale * v);
      wf[hi + per_layer] = P::to_w_lo(scale * v);
    }
  }
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid < nW * F) reinterpret_cast<Acc*>(bias)[tid] = (Acc)(scale * b[tid]);
  if (tid < 2 * F) {
    const int x = tid / F, f = tid % F;
    double h;
    if (act == 0) {
      h = tanh(We[x * F + f] + be[f]);
    } else {
      double mu = 0.0, var = 0.0;
      for (int g = 0; g < F; ++g) mu += fmax(We[x * F + g] + be[g], 0.0);
      mu /= F;
      for (int g = 0; g < F; ++g) {
        const double d = fmax(We[x * F + g] + be[g], 0.0) - mu;
        var += d * d;
      }
      var /= F;
      h = (fmax(We[x * F + f] + be[f], 0.0) - mu) / sqrt(var + kLnEps);
    }
    reinterpret_cast<Acc*>(emb)[tid] = (Acc)h;
  }
}

template <class P, int F, int TPW, int NCH>
__global__ __launch_bounds__(512) void k_logpsi(Net net, const int8_t* __restrict__ spins, int B,
                                                 double* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  Smem<P> s(net.g, smem);
  stage_graph<P>(net, s);
  if (net.tied) stage_weights<P, F>(net, s, 0);
  __syncthreads();
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    load_spins<P>(net, s, spins + (size_t)b * net.n);
    double la = 0, ph = 0;
    eval_config<P, F, TPW, NCH>(net, s, -1, -1, la, ph);
    if (threadIdx.x == 0) {
      out[2 * (size_t)b] = la;
      out[2 * (size_t)b + 1] = ph;
    }
  }
}

__device__ __forceinline__ void neumaier(double& sum, double& comp, double x) {
  const double t = sum + x;
  comp += (fabs(sum) >= fabs(x)) ? ((sum - t) + x) : ((x - t) + sum);
  sum = t;
}

// partial[item] = {sum re, comp re, sum im, comp im} of psi(s^ij)/psi(s) over the
// anti-aligned bonds of chunk c of sample b (item = b * n_chunks + c), in bond order.
template <class P, int F, int TPW, int NCH>
__global__ __launch_bounds__(512) void k_eloc(Net net, const int8_t* __restrict__ spins, int B,
                                               const double* __restrict__ base, int n_chunks, int chunk,
                                               double* __restrict__ partial, int* __restrict__ cnt) {
  extern __shared__ __align__(16) unsigned char smem[];
  Smem<P> s(net.g, smem);
  stage_graph<P>(net, s);
  if (net.tied) stage_weights<P, F>(net, s, 0);
  __syncthreads();
  const int items = B * n_chunks;
  for (int it = blockIdx.x; it < items; it += gridDim.x) {
    const int b = it / n_chunks, c = it % n_chunks;
    load_spins<P>(net, s, spins + (size_t)b * net.n);
    const double lb = base[2 * (size_t)b], pb = base[2 * (size_t)b + 1];
    double sr = 0, cr = 0, si = 0, ci = 0;
    int ne = 0;
    const int e0 = c * chunk, e1 = min(net.ne, e0 + chunk);
    for (int e = e0; e < e1; ++e) {
      const int2 ij = net.edges[e];
      if (s.sp[ij.x] == s.sp[ij.y]) continue;   // uniform across the workgroup
      double la = 0, ph = 0;
      eval_config<P, F, TPW, NCH>(net, s, ij.x, ij.y, la, ph);
      if (threadIdx.x == 0) {
        const double m = exp(la - lb);
        double sn, cs;
        sincos(ph - pb, &sn, &cs);
        neumaier(sr, cr, m * cs);
        neumaier(si, ci, m * sn);
        ++ne;
      }
    }
    if (threadIdx.x == 0) {
      double* o = partial + 4 * (size_t)it;
      o[0] = sr; o[1] = cr; o[2] = si; o[3] = ci;
      cnt[it] = ne;
    }
    __syncthreads();
  }
}

__global__ void k_zero_i64(long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// device-resident Philox counter base of the sampler: advanced by each step
__global__ void k_add_u64(unsigned long long* p, unsigned long long d) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += d;
}

// Per-item sums of the pipelined local energy's exchange terms (Section 3's E_x:
// psi(s^ij) / psi(s) = exp(da + i dp) for each anti-aligned bond of the item, with
// (da, dp) = terms[b][e]), compensated and in bond order: the order in which the
// kernels that sum in place take them.
__global__ void k_eloc_terms(const int8_t* __restrict__ spins, int N, const int2* __restrict__ edges, int E,
                             int B, int n_chunks, int chunk, const double* __restrict__ terms,
                             double* __restrict__ partial, int* __restrict__ cnt) {
  const long long item = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= (long long)B * n_chunks) return;
  const int b = (int)(item / n_chunks), cc = (int)(item % n_chunks);
  const int e0 = cc * chunk, e1 = min(E, e0 + chunk);
  const int8_t* sb = spins + (size_t)b * N;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int n = 0;
  for (int e = e0; e < e1; ++e) {
    const int2 ij = edges[e];
    if (sb[ij.x] == sb[ij.y]) continue;
    const double* o = terms + 2 * ((size_t)b * E + e);
    const double mm = exp(o[0]);
    double sn, cs;
    sincos(o[1], &sn, &cs);
    inc_neumaier(a0, a1, mm * cs);
    inc_neumaier(a2, a3, mm * sn);
    ++n;
  }
  double* p = partial + 4 * item;
  p[0] = a0;
  p[1] = a1;
  p[2] = a2;
  p[3] = a3;
  cnt[item] = n;
}

// log psi of each chain from the layer-L readout partials that its planes hold (the
// incremental base pass writes them and the incremental sampler keeps them current):
// the sum of the full evaluation, replayed in its order -- each lane adds its tiles'
// partials in tile order, the wave sums its lanes (wave_sum), the waves' sums are
// added in wave order, then the spin-count terms -- so the result is bitwise the
// full evaluation's.  One wave per chain.
__global__ void k_logpsi_planes(const unsigned char* __restrict__ planes, size_t per_bytes, size_t part_off,
                                const int8_t* __restrict__ spins, int N, int B, int wpc, int tpw, int F,
                                const double* __restrict__ head_a, const double* __restrict__ head_p,
                                double* __restrict__ out) {
  const int lane = threadIdx.x & 63, col = lane & 15, q = lane >> 4;
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (b >= B) return;
  const double* part = reinterpret_cast<const double*>(planes + (size_t)b * per_bytes + part_off);
  double a = 0.0, p = 0.0;
  for (int w = 0; w < wpc; ++w) {
    double pa = 0.0, pp = 0.0;
    for (int k = 0; k < tpw; ++k) {
      const int node = (w + k * wpc) * 16 + col;
      if (node < N) {
        pa += part[(size_t)node * 8 + q * 2];
        pp += part[(size_t)node * 8 + q * 2 + 1];
      }
    }
    pa = wave_sum(pa);
    pp = wave_sum(pp);
    a += pa;
    p += pp;
  }
  const int8_t* sb = spins + (size_t)b * N;
  int c = 0;
  for (int k = lane; k < N; k += 64) c += sb[k] > 0 ? 1 : 0;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
  if (lane == 0) {
    const double nup = (double)c, ndn = (double)N - nup;
    a += head_a[F] * ndn + head_a[F + 1] * nup + head_a[F + 2];
    p += head_p[F] * ndn + head_p[F + 1] * nup + head_p[F + 2];
    out[2 * (size_t)b] = a;
    out[2 * (size_t)b + 1] = p;
  }
}

__global__ void k_eloc_finalize(const int8_t* __restrict__ spins, int N, const int2* __restrict__ edges,
                                int E, double jz, double jxy, double hb, double cb, int B, int n_chunks,
                                const double* __restrict__ partial, const int* __restrict__ cnt,
                                double* __restrict__ eloc, long long* n_evals) {
  // one wave per sample: its lanes split the bonds of the diagonal and field sums
  // (integers, exact in any order); lane 0 adds the exchange part
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (b >= B) return;
  const int8_t* sb = spins + (size_t)b * N;
  long long diag = 0, field = 0;
  for (int e = lane; e < E; e += 64) {
    const int2 ij = edges[e];
    const int si = sb[ij.x], sj = sb[ij.y];
    diag += si * sj;
    field += si + sj;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    diag += __shfl_xor(diag, o, 64);
    field += __shfl_xor(field, o, 64);
  }
  if (lane != 0) return;
  double sr = 0, cr = 0, si = 0, ci = 0;
  long long ne = 1;
  for (int c = 0; c < n_chunks; ++c) {
    const double* o = partial + 4 * ((size_t)b * n_chunks + c);
    neumaier(sr, cr, o[0]);
    cr += o[1];
    neumaier(si, ci, o[2]);
    ci += o[3];
    ne += cnt[(size_t)b * n_chunks + c];
  }
  eloc[2 * (size_t)b] = 0.25 * jz * (double)diag + 0.25 * hb * (double)field + cb * (double)E + 0.5 * jxy * (sr + cr);
  eloc[2 * (size_t)b + 1] = 0.5 * jxy * (si + ci);
  if (n_evals) atomicAdd(reinterpret_cast<unsigned long long*>(n_evals), (unsigned long long)ne);
}

template <class P, int F, int TPW, int NCH>
__global__ __launch_bounds__(512) void k_sweep(Net net, int8_t* __restrict__ spins, double* __restrict__ logpsi,
                                                int B, int n_sweeps, unsigned long long seed,
                                                unsigned long long counter_base,
                                                const unsigned long long* __restrict__ counter_dev,
                                                int* __restrict__ n_accept) {
  extern __shared__ __align__(16) unsigned char smem[];
  Smem<P> s(net.g, smem);
  if (counter_dev) counter_base += *counter_dev;   // graph replays read the current base
  stage_graph<P>(net, s);
  if (net.tied) stage_weights<P, F>(net, s, 0);
  __syncthreads();
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const long long total = (long long)n_sweeps * net.n;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    load_spins<P>(net, s, spins + (size_t)b * net.n);
    double lr = logpsi[2 * (size_t)b], li = logpsi[2 * (size_t)b + 1];
    int acc = 0;
    for (long long t = 0; t < total; ++t) {
      const unsigned long long step = counter_base + (unsigned long long)t;
      uint32_t c[4] = {(uint32_t)step, (uint32_t)(step >> 32), (uint32_t)b, 0u};
      philox4x32_10(c, k0, k1);
      const int e = (int)(((unsigned long long)c[0] * (unsigned long long)net.ne) >> 32);
      const double u = ((double)c[1] + 0.5) * 2.3283064365386963e-10;   // 2^-32
      const int2 ij = net.edges[e];
      if (s.sp[ij.x] == s.sp[ij.y]) continue;                             // identity step
      double la = 0, ph = 0;
      eval_config<P, F, TPW, NCH>(net, s, ij.x, ij.y, la, ph);
      if (threadIdx.x == 0) {
        if (u < exp(2.0 * (la - lr))) {
          const int8_t tmp = s.sp[ij.x];
          s.sp[ij.x] = s.sp[ij.y];
          s.sp[ij.y] = tmp;
          lr = la;
          li = ph;
          ++acc;
        }
      }
      __syncthreads();
    }
    for (int k = threadIdx.x; k < net.n; k += blockDim.x) spins[(size_t)b * net.n + k] = s.sp[k];
    if (threadIdx.x == 0) {
      logpsi[2 * (size_t)b] = lr;
      logpsi[2 * (size_t)b + 1] = li;
      if (n_accept) n_accept[b] = acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// ISGO statistics (single workgroup of 1024 threads, FP64, fixed reduction order)
// ---------------------------------------------------------------------------
constexpr int kStatThreads = 1024;

__device__ void two_sum_merge(double& s, double& c, double s2, double c2) {
  const double t = s + s2;
  const double e = (fabs(s) >= fabs(s2)) ? ((s - t) + s2) : ((s2 - t) + s);
  s = t;
  c = c + c2 + e;
}

// block-wide compensated sum of (s, c) pairs; result valid in thread 0
__device__ double block_sum(double s, double c, double* sh_s, double* sh_c) {
  const int tid = threadIdx.x;
  sh_s[tid] = s;
  sh_c[tid] = c;
  __syncthreads();
  for (int st = kStatThreads / 2; st > 0; st >>= 1) {
    if (tid < st) {
      double a = sh_s[tid], ac = sh_c[tid];
      two_sum_merge(a, ac, sh_s[tid + st], sh_c[tid + st]);
      sh_s[tid] = a;
      sh_c[tid] = ac;
    }
    __syncthreads();
  }
  const double r = sh_s[0] + sh_c[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kStatThreads) void k_isgo_stats(
    int B, const double* __restrict__ lp_old, const double* __restrict__ lp_new,
    const double* __restrict__ eloc, const double* __restrict__ counts, const long long* __restrict__ n_evals,
    double* __restrict__ stats, double* __restrict__ cot) {
  __shared__ double sh_s[kStatThreads], sh_c[kStatThreads];
  __shared__ double bc[8];
  const int tid = threadIdx.x;
  const int per = (B + kStatThreads - 1) / kStatThreads;
  const int a0 = min(B, tid * per), a1 = min(B, a0 + per);
  // 1. max shift and finiteness
  double mloc = -INFINITY;
  int bad = 0;
  for (int x = a0; x < a1; ++x) {
    const double d = 2.0 * (lp_new[2 * x] - lp_old[2 * x]);
    const double n = counts ? counts[x] : 1.0;
    if (!isfinite(d) || !isfinite(eloc[2 * x]) || !isfinite(eloc[2 * x + 1]) || !isfinite(n)) bad = 1;
    mloc = fmax(mloc, d);
  }
  sh_s[tid] = mloc;
  sh_c[tid] = (double)bad;
  __syncthreads();
  for (int st = kStatThreads / 2; st > 0; st >>= 1) {
    if (tid < st) {
      sh_s[tid] = fmax(sh_s[tid], sh_s[tid + st]);
      sh_c[tid] = fmax(sh_c[tid], sh_c[tid + st]);
    }
    __syncthreads();
  }
  const double m = (B > 0) ? sh_s[0] : 0.0;
  const double nonfinite = sh_c[0];
  __syncthreads();
  // 2. sums of r, r E, r^2
  double s0 = 0, c0 = 0, sre = 0, cre = 0, sim = 0, cim = 0, sq = 0, cq = 0;
  for (int x = a0; x < a1; ++x) {
    const double n = counts ? counts[x] : 1.0;
    const double r = n * exp(2.0 * (lp_new[2 * x] - lp_old[2 * x]) - m);
    neumaier(s0, c0, r);
    neumaier(sre, cre, r * eloc[2 * x]);
    neumaier(sim, cim, r * eloc[2 * x + 1]);
    neumaier(sq, cq, r * r);
  }
  const double S = block_sum(s0, c0, sh_s, sh_c);
  const double SR = block_sum(sre, cre, sh_s, sh_c);
  const double SI = block_sum(sim, cim, sh_s, sh_c);
  const double Q = block_sum(sq, cq, sh_s, sh_c);
  if (tid == 0) {
    bc[0] = S;
    bc[1] = SR / S;
    bc[2] = SI / S;
  }
  __syncthreads();
  const double Ssum = bc[0], er = bc[1], ei = bc[2];
  // 3. variance and cotangents
  double sv = 0, cv = 0;
  for (int x = a0; x < a1; ++x) {
    const double n = counts ? counts[x] : 1.0;
    const double r = n * exp(2.0 * (lp_new[2 * x] - lp_old[2 * x]) - m);
    const double p = r / Ssum;
    const double dr = eloc[2 * x] - er, di = eloc[2 * x + 1] - ei;
    neumaier(sv, cv, r * (dr * dr + di * di));
    cot[2 * x] = 2.0 * p * dr;
    cot[2 * x + 1] = 2.0 * p * di;
  }
  const double V = block_sum(sv, cv, sh_s, sh_c);
  if (tid == 0) {
    const bool empty = (B == 0);
    stats[0] = empty ? 0.0 : er;
    stats[1] = empty ? 0.0 : ei;
    stats[2] = empty ? 0.0 : V / Ssum;
    stats[3] = empty ? 0.0 : Ssum * Ssum / Q;
    stats[4] = Ssum;
    stats[5] = m;
    stats[6] = n_evals ? (double)n_evals[0] : 0.0;
    stats[7] = nonfinite;
  }
}

__global__ void k_vjp_reduce(const double* __restrict__ part, int nrows, int npar, double* __restrict__ grad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npar) return;
  double s = 0.0, c = 0.0;
  // rows in order; 32 of them requested at a time
  int r = 0;
  for (; r + 32 <= nrows; r += 32) {
    double x[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) x[u] = part[(size_t)(r + u) * npar + k];
#pragma unroll
    for (int u = 0; u < 32; ++u) neumaier(s, c, x[u]);
  }
  for (; r < nrows; ++r) neumaier(s, c, part[(size_t)r * npar + k]);
  grad[k] = s + c;
}

__global__ void k_sgd(double* theta, const double* grad, double alpha, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) theta[k] -= alpha * grad[k];
}

__global__ void k_fill(double* p, double v, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

// ---------------------------------------------------------------------------
// Grouping of duplicated states into unique states with counts (Section 3).
// Each row is packed 64 sites per wave ballot and hashed; an open-addressing
// table keyed by the hash keeps the smallest row index per key, and a row whose
// contents equal that row's joins its group.  Groups are numbered in the order of
// their first rows, so the output is the rows' first-occurrence order.
// ---------------------------------------------------------------------------
// splitmix64 output function (Steele, Lea and Flood, OOPSLA 2014) as the mixer
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_group_clear(unsigned long long* __restrict__ keys, int* __restrict__ vals, int T,
                              int* __restrict__ cnt, int B) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < T; i += gridDim.x * blockDim.x) {
    keys[i] = 0ull;
    vals[i] = 0x7FFFFFFF;
    if (i < B) cnt[i] = 0;
  }
}

// one wave per row; T is a power of two >= 2B, so a free slot always exists
__global__ void k_group_insert(const int8_t* __restrict__ spins, int n, int B, unsigned long long* keys,
                               int* vals, int T, int* __restrict__ slot_of) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (b >= B) return;   // wave-uniform
  const int8_t* sb = spins + (size_t)b * n;
  unsigned long long h = 0x9E3779B97F4A7C15ull ^ (unsigned long long)n;
  for (int c = 0; c < n; c += 64) {
    const bool up = (c + lane < n) && sb[c + lane] > 0;
    h = mix64(h ^ (unsigned long long)__ballot(up)) + (unsigned long long)c;
  }
  if (h == 0ull) h = 1ull;   // 0 marks a free slot
  if (lane == 0) {
    int slot = (int)(h & (unsigned long long)(T - 1)), found = -1;
    for (int probe = 0; probe < T; ++probe) {
      const unsigned long long prev = atomicCAS(&keys[slot], 0ull, h);
      if (prev == 0ull || prev == h) {
        atomicMin(&vals[slot], b);
        found = slot;
        break;
      }
      slot = (slot + 1) & (T - 1);
    }
    slot_of[b] = found;
  }
}

// rep[b]: the group's first row, or b itself when the rows differ (a hash collision)
__global__ void k_group_rep(const int8_t* __restrict__ spins, int n, int B, const int* __restrict__ vals,
                            const int* __restrict__ slot_of, int* __restrict__ rep) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (b >= B) return;
  const int slot = slot_of[b];
  int r = slot >= 0 ? vals[slot] : b;
  if (r != b) {
    const int8_t* x = spins + (size_t)b * n;
    const int8_t* y = spins + (size_t)r * n;
    bool diff = false;
    for (int i = lane; i < n; i += 64) diff |= (x[i] != y[i]);
    if (__ballot(diff) != 0ull) r = b;
  }
  if (lane == 0) rep[b] = r;
}

// gid[b] = number of first rows before b (one workgroup of 1024 threads)
__global__ __launch_bounds__(1024) void k_group_scan(const int* __restrict__ rep, int B, int* __restrict__ gid,
                                                     int* __restrict__ n_unique) {
  __shared__ int s_w[16];
  __shared__ int s_base;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < B; c0 += 1024) {
    const int b = c0 + threadIdx.x;
    const bool head = b < B && rep[b] == b;
    const unsigned long long m = __ballot(head);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_w[wv] = __popcll(m);
    __syncthreads();
    int off = s_base;
    for (int k = 0; k < wv; ++k) off += s_w[k];
    if (b < B) gid[b] = off + before;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int k = 0; k < 16; ++k) t += s_w[k];
      s_base += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_unique = s_base;
}

// one wave per row: count it into its group; a first row is copied to its slot
__global__ void k_group_scatter(const int8_t* __restrict__ spins, int n, int B, const int* __restrict__ rep,
                                const int* __restrict__ gid, int* cnt, int8_t* __restrict__ uniq) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (b >= B) return;
  const int r = rep[b], g = gid[r];
  if (lane == 0) atomicAdd(&cnt[g], 1);
  if (r == b) {
    const int8_t* x = spins + (size_t)b * n;
    int8_t* y = uniq + (size_t)g * n;
    for (int i = lane; i < n; i += 64) y[i] = x[i];
  }
}

// counts as FP64; rows past the unique ones repeat the first unique row with count 0
__global__ void k_group_finish(const int* __restrict__ cnt, const int* __restrict__ n_unique, int n, int B,
                               double* __restrict__ counts, int8_t* __restrict__ uniq) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= B) return;
  const int U = *n_unique;
  if (p < U) {
    if (lane == 0) counts[p] = (double)cnt[p];
    return;
  }
  if (lane == 0) counts[p] = 0.0;
  for (int i = lane; i < n; i += 64) uniq[(size_t)p * n + i] = uniq[i];
}

// ===========================================================================
// Host side
// ===========================================================================

std::mutex g_err_mu;
std::string g_init_err;

struct Kern {  // kernels of one (precision, F, TPW, NCH) instantiation
  const void* logpsi = nullptr;
  const void* eloc = nullptr;
  const void* sweep = nullptr;
  void (*prepare)(const double*, int, int, void*, void*, void*, hipStream_t) = nullptr;
};

template <class P, int F, int TPW, int NCH>
Kern make_kern() {
  Kern k;
  k.logpsi = reinterpret_cast<const void*>(&k_logpsi<P, F, TPW, NCH>);
  k.eloc = reinterpret_cast<const void*>(&k_eloc<P, F, TPW, NCH>);
  k.sweep = reinterpret_cast<const void*>(&k_sweep<P, F, TPW, NCH>);
  k.prepare = [](const double* th, int nW, int act, void* wf, void* bias, void* emb, hipStream_t st) {
    const int total = nW * 2 * F * F;
    const int blocks = std::max(1, std::min(1024, (total + 255) / 256));
    hipLaunchKernelGGL((k_prepare<P, F>), dim3(blocks), dim3(256), 0, st, th, nW, act, wf, bias, emb);
  };
  return k;
}

template <class P, int F, int NCH>
Kern pick_tpw(int tpw) {
  switch (tpw) {
    case 1: return make_kern<P, F, 1, NCH>();
    case 2: return make_kern<P, F, 2, NCH>();
    default: return make_kern<P, F, 4, NCH>();
  }
}

template <class P, int F>
Kern pick_nch(int tpw, int nch) {
  if constexpr ((F / 16) % 4 == 0) {
    if (nch == 4) return pick_tpw<P, F, 4>(tpw);
  }
  return pick_tpw<P, F, 1>(tpw);
}

template <class P>
Kern pick_f(int F, int tpw, int nch) {
  if (F == 16) return pick_nch<P, 16>(tpw, nch);
  if (F == 32) return pick_nch<P, 32>(tpw, nch);
  return pick_nch<P, 64>(tpw, nch);
}

// incremental local energy: base pass (precision, F, TPW, NCH) and ball kernel (precision, F, MAXT)
template <class P, int F, int TPW, int NCH>
const void* inc_base_kernel() {
  return reinterpret_cast<const void*>(&k_inc_base<P, F, TPW, NCH>);
}
template <class P, int F>
const void* inc_base_pick(int tpw, int nch) {
  if constexpr ((F / 16) % 4 == 0) {
    if (nch == 4) {
      if (tpw == 1) return inc_base_kernel<P, F, 1, 4>();
      if (tpw == 2) return inc_base_kernel<P, F, 2, 4>();
      return inc_base_kernel<P, F, 4, 4>();
    }
  }
  if (tpw == 1) return inc_base_kernel<P, F, 1, 1>();
  if (tpw == 2) return inc_base_kernel<P, F, 2, 1>();
  return inc_base_kernel<P, F, 4, 1>();
}
struct IncKern {
  const void* base = nullptr;    // k_inc_base
  const void* eloc = nullptr;    // k_eloc_inc
  const void* sweep = nullptr;   // k_sweep_inc
};
template <class P, int F, int MAXT, int NT = 512>
void inc_fill(IncKern& k) {
  k.eloc = reinterpret_cast<const void*>(&k_eloc_inc<P, F, MAXT, NT>);
  k.sweep = reinterpret_cast<const void*>(&k_sweep_inc<P, F, MAXT, NT>);
}
template <class P, int F>
IncKern inc_pick(int tpw, int nch, int maxt, bool wide) {
  IncKern k;
  k.base = inc_base_pick<P, F>(tpw, nch);
  if (wide) inc_fill<P, F, 1, 1024>(k);   // 16 waves, one tile each
  else if (maxt == 1) inc_fill<P, F, 1>(k);
  else if (maxt == 2) inc_fill<P, F, 2>(k);
  else if (maxt == 3) inc_fill<P, F, 3>(k);
  else inc_fill<P, F, 4>(k);
  return k;
}
template <class P>
IncKern inc_pick_f(int F, int tpw, int nch, int maxt, bool wide) {
  if (F == 16) return inc_pick<P, 16>(tpw, nch, maxt, wide);
  if (F == 32) return inc_pick<P, 32>(tpw, nch, maxt, wide);
  return inc_pick<P, 64>(tpw, nch, maxt, wide);
}

// reverse-pass kernels of one (precision, F, TPW, NCH) instantiation (FP32 or FP64)
struct VKern {
  const void* fwd = nullptr;
  const void* dx = nullptr;
  const void* dw = nullptr;
  const void* tail = nullptr;
  Kern fk{};   // forward kernels of the same precision (prepare)
  void (*prepare_bwd)(const double*, int, void*, hipStream_t) = nullptr;
};

template <class P, int F, int TPW, int NCH>
VKern make_vkern() {
  VKern k;
  k.fwd = reinterpret_cast<const void*>(&k_vjp_fwd<P, F, TPW, NCH>);
  k.dx = reinterpret_cast<const void*>(&k_vjp_dx<P, F, TPW>);
  k.dw = reinterpret_cast<const void*>(&k_vjp_dw<P, F>);
  k.tail = reinterpret_cast<const void*>(&k_vjp_tail<P, F>);
  k.fk = make_kern<P, F, TPW, NCH>();
  k.prepare_bwd = [](const double* th, int nW, void* out, hipStream_t st) {
    const int total = nW * 2 * F * F;
    const int blocks = std::max(1, std::min(1024, (total + 255) / 256));
    hipLaunchKernelGGL((k_prepare_bwd<P, F>), dim3(blocks), dim3(256), 0, st, th, nW,
                       reinterpret_cast<typename P::Acc*>(out));
  };
  return k;
}

template <class P, int F, int NCH>
VKern vpick_tpw(int tpw) {
  switch (tpw) {
    case 1: return make_vkern<P, F, 1, NCH>();
    case 2: return make_vkern<P, F, 2, NCH>();
    default: return make_vkern<P, F, 4, NCH>();
  }
}

template <class P, int F>
VKern vpick_nch(int tpw, int nch) {
  if constexpr ((F / 16) % 4 == 0) {
    if (nch == 4) return vpick_tpw<P, F, 4>(tpw);
  }
  return vpick_tpw<P, F, 1>(tpw);
}

template <class P>
VKern vpick_f(int F, int tpw, int nch) {
  if (F == 16) return vpick_nch<P, 16>(tpw, nch);
  if (F == 32) return vpick_nch<P, 32>(tpw, nch);
  return vpick_nch<P, 64>(tpw, nch);
}

}  // namespace

struct gna_ctx {
  int N = 0, E = 0, F = 0, L = 0, tied = 1, prec = 0, max_batch = 0;
  double jz = 1.0, jxy = 1.0, hb = 0.0, cb = 0.0;   // bond Hamiltonian (gna_set_couplings)
  hipStream_t stream = nullptr;
  int device = 0, n_cu = 0;
  int64_t P = 0;
  std::string err;
  // geometry
  int tpw = 1, nch = 1, dmax = 1;
  Geo geo{};
  Kern kern{};
  int grid_logpsi = 1, grid_eloc = 1, grid_sweep = 1;
  int max_chunks = 1;
  size_t sz_W = 8, sz_Acc = 8;
  // device buffers
  int2* d_edges = nullptr;
  int* d_idx = nullptr;
  void* d_val = nullptr;       // Acc precision
  double* d_val64 = nullptr;   // FP64 A_hat for the reverse pass
  void* d_wfrag = nullptr;
  void* d_bias = nullptr;
  void* d_emb = nullptr;
  double* d_base = nullptr;     // [max_batch][2]
  double* d_partial = nullptr;  // [max_batch * max_chunks][4]
  int* d_cnt = nullptr;         // [max_batch * max_chunks]
  long long* d_nev = nullptr;   // [1]
  double* d_cot = nullptr;      // [max_batch][2]
  double* d_eloc = nullptr;     // [max_batch][2]
  unsigned long long* d_grp_key = nullptr;   // [grp_T] row hashes (0: free)
  int* d_grp_val = nullptr;     // [grp_T] smallest row index per hash
  int* d_grp_row = nullptr;     // [4][max_batch]: slot, first row, group id, count
  int grp_T = 0;                // power of two >= 2 max_batch
  // incremental local energy
  int eloc_mode = 0;
  IncGeo igeo{};
  IncKern ik{};
  int grid_inc_base = 1, grid_inc = 1, grid_sweep_inc = 1, inc_r8 = 8, inc_chunk_cap = 64;
  bool inc_wide = false;   // 16-wave incremental kernels
  IncGeo igeo_sw{};        // shape of the incremental sweep kernel (tuned on its own)
  bool inc_sw_wide = false;
  int inc_sw_maxt = 1;
  int inc_per_xcd = 2;     // samples in flight per XCD (local energy work items)
  int inc_maxt = 1;        // tiles per wave
  int inc_max_rows = 2, inc_max_ball = 2, inc_max_tiles = 1;
  size_t inc_w_bytes = 0, lds_max = 0;
  std::string tune_key;    // shape signature for the tuner's cache
  int2* d_ball_meta = nullptr;
  int* d_ball_cnt = nullptr;
  uint16_t* d_ball_tab = nullptr;
  void* d_inc_planes = nullptr;   // [max_batch][2L][npad][F] Acc
  // layer-pipelined incremental kernels (gna_pipe.h)
  bool pipe_ok = false;            // its bond tables exist (sizes within the 12-bit pool tags)
  bool pipe_el = false, pipe_sw = false;   // the local energy / the sweep run pipelined
  bool split_w = false;                    // BF16 weights as hi + lo pairs (PBF16S)
  PipeGeo pgeo_el{}, pgeo_sw{};
  PipeKern pk_el{}, pk_sw{};
  int grid_pipe_el = 1, grid_pipe_sw = 1;
  int pipe_tabw = 0;
  std::vector<int> ball_cmax;      // max |C_l| over bonds, l = 0 .. L+1
  std::vector<int> ball_ringmax;   // max |C_s| - |C_{s-1}| over bonds, s = 3 .. L+1 (index s)
  uint2* d_sched = nullptr;        // [2][kPipeMaxD][kMaxWaves] tile schedules: local energy, sweep
  uint16_t* d_pipe_tab = nullptr;  // per bond: header, node ids, pool tags of positions and neighbours
  double* d_terms = nullptr;       // pipelined local energy: [max_batch][E][2] exchange readout differences
  // reverse pass (FP32 for the FP32/BF16 modes, FP64 for FP64)
  Geo vgeo{};
  VKern vk{};
  int vgrid_fwd = 1, vgrid_dx = 1, vjp_rows = 1;
  size_t vdx_lds = 0;   // k_vjp_dx: one layer's backward fragments and the adjacency
  void* d_vwfrag = nullptr;
  void* d_vbias = nullptr;
  void* d_vemb = nullptr;
  void* d_wbwd = nullptr;
  void* d_planes = nullptr;     // [vjp_chunk][nplanes][npad][F] Acc
  int vjp_chunk = 1, nplanes = 1;
  int act = 0;                  // GNA_ACT_*
  double* d_vjp_part = nullptr; // [vjp_rows][P]
  std::vector<void*> owned;
  void* scratch_dev = nullptr;  // this device's copy of `scratch` (hipGetSymbolAddress), or NULL
  std::string scratch_err;      // why scratch_dev is NULL
  // kernel timing (gna_profile_enable)
  bool prof_on = false;
  bool prof_err = false;        // an event could not be created or recorded since the last read
  struct Rec { const char* name; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

gna_status fail(gna_ctx* c, gna_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

gna_status hip_fail(gna_ctx* c, hipError_t e, const char* what) {
  return fail(c, GNA_HIP_ERROR, std::string(what) + ": " + hipGetErrorString(e));
}

#define GNA_HIP(ctx, call)                                      \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);    \
  } while (0)

// Device address of `scratch` on `device` (the current device), looked up once per
// device and kept for the process.
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_dev[kMaxDevices] = {};

hipError_t static_scratch(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

hipEvent_t take_event(gna_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Scope guard recording start/stop events around one launch when timing is on.  A
// failed event creation or record drops the launch from the record and marks it
// (gna_profile_read then reports the failure instead of partial timings).
struct Timed {
  gna_ctx* c;
  const char* name;
  hipEvent_t a = nullptr;
  Timed(gna_ctx* c_, const char* n) : c(c_), name(n) {
    if (!c->prof_on) return;
    a = take_event(c);
    if (!a) {
      c->prof_err = true;
    } else if (hipEventRecord(a, c->stream) != hipSuccess) {
      c->ev_pool.push_back(a);
      a = nullptr;
      c->prof_err = true;
    }
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b || hipEventRecord(b, c->stream) != hipSuccess) {
      c->ev_pool.push_back(a);
      if (b) c->ev_pool.push_back(b);
      c->prof_err = true;
      return;
    }
    c->recs.push_back({name, a, b});
  }
};

template <class X>
gna_status dev_alloc(gna_ctx* c, X** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return fail(c, GNA_OUT_OF_MEMORY, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  c->owned.push_back(q);
  *p = reinterpret_cast<X*>(q);
  return GNA_OK;
}

void free_all(gna_ctx* c) {
  for (void* p : c->owned) (void)hipFree(p);   // teardown: nothing to report to
  c->owned.clear();
}

int64_t param_count(int F, int L, int tied) {
  const int64_t nW = tied ? 1 : L;
  return 2LL * F + F + nW * (2LL * F * F + F) + 2LL * (F + 3);
}

gna_status check_launch(gna_ctx* c, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, what);
  return GNA_OK;
}

gna_status prepare(gna_ctx* c, const double* theta) {
  Timed tm(c, "k_prepare");
  c->kern.prepare(theta, c->tied ? 1 : c->L, c->act, c->d_wfrag, c->d_bias, c->d_emb, c->stream);
  return check_launch(c, "k_prepare");
}

Net make_net(gna_ctx* c, const double* theta) {
  Net n{};
  n.n = c->N;
  n.ne = c->E;
  n.F = c->F;
  n.L = c->L;
  n.tied = c->tied;
  n.act = c->act;
  n.dmax = c->dmax;
  n.ell_idx = c->d_idx;
  n.ell_val = c->d_val;
  n.edges = c->d_edges;
  n.wfrag = c->d_wfrag;
  n.bias = c->d_bias;
  n.emb = c->d_emb;
  const int nW = c->tied ? 1 : c->L;
  n.head_a = theta + 3 * c->F + (size_t)nW * (2 * c->F * c->F + c->F);
  n.head_p = n.head_a + c->F + 3;
  n.g = c->geo;
  return n;
}

gna_status launch(gna_ctx* c, const void* fn, int grid, void** args, const char* what) {
  Timed tm(c, what);
  hipError_t e = hipLaunchKernel(fn, dim3(grid), dim3(64 * c->geo.wpc), args, (size_t)c->geo.lds_bytes, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, what);
  return check_launch(c, what);
}

gna_status run_logpsi(gna_ctx* c, const double* theta, const int8_t* spins, int B, double* out) {
  if (B == 0) return GNA_OK;
  Net net = make_net(c, theta);
  int grid = std::min(B, c->grid_logpsi);
  void* args[] = {&net, &spins, &B, &out};
  return launch(c, c->kern.logpsi, grid, args, "k_logpsi");
}

// log psi of the chains whose planes hold their current base pass (after the
// incremental sampler), read from the readout partials; bitwise run_logpsi's result
gna_status run_logpsi_planes(gna_ctx* c, const double* theta, const int8_t* spins, int B, double* out) {
  if (B == 0) return GNA_OK;
  if (c->L < 1) return run_logpsi(c, theta, spins, B, out);
  const size_t plane = (size_t)c->geo.npad * c->F;
  const size_t per_bytes = (size_t)2 * c->L * plane * c->sz_Acc;
  const size_t part_off = (size_t)(c->L - 1) * plane * c->sz_Acc;
  const Net net = make_net(c, theta);
  Timed tm(c, "k_logpsi_planes");
  hipLaunchKernelGGL(k_logpsi_planes, dim3((B + 3) / 4), dim3(256), 0, c->stream,
                     reinterpret_cast<const unsigned char*>(c->d_inc_planes), per_bytes, part_off, spins, c->N, B,
                     c->geo.wpc, c->tpw, c->F, net.head_a, net.head_p, out);
  return check_launch(c, "k_logpsi_planes");
}

IncNet make_inc(const gna_ctx* c) {
  IncNet inc{};
  inc.n = c->N; inc.F = c->F; inc.L = c->L; inc.dmax = c->dmax; inc.r8 = c->inc_r8;
  inc.ball_meta = c->d_ball_meta; inc.ball_cnt = c->d_ball_cnt; inc.ball_tab = c->d_ball_tab;
  inc.ell_val = c->d_val;
  return inc;
}

// Bond chunks of the local energy's work items (item = sample x chunk of bonds):
// enough items to balance the persistent grid, at most c->max_chunks per sample.
void eloc_chunks(const gna_ctx* c, int B, int* n_chunks_out, int* chunk_out) {
  const long long work = (long long)B * std::max(1, c->E);
  long long chunk = work / (16LL * c->grid_eloc);
  chunk = std::max<long long>(16, std::min<long long>(chunk, std::max(1, c->E)));
  if (c->eloc_mode == GNA_ELOC_INCREMENTAL) {
    // inc_per_xcd samples per XCD at a time: per_x / inc_per_xcd chunks per sample;
    // a chunk holds at most one bond per thread of the workgroup
    const int per_x = std::max(1, c->grid_inc / 8);
    const int per_sample = std::max(1, per_x / c->inc_per_xcd);
    chunk = std::max<long long>(8, (std::max(1, c->E) + per_sample - 1) / per_sample);
    chunk = std::min<long long>(chunk, c->inc_chunk_cap);
  }
  int n_chunks = (int)((std::max(1, c->E) + chunk - 1) / chunk);
  if (n_chunks > c->max_chunks) {
    n_chunks = c->max_chunks;
    chunk = (c->E + n_chunks - 1) / n_chunks;
  }
  *n_chunks_out = n_chunks;
  *chunk_out = (int)chunk;
}

// planes_ready (incremental mode): the planes and `base` already hold the base pass
// of exactly these configurations under this theta (an incremental sweep just left
// them so), and the base pass is skipped.  partial / cnt: per-item scratch of at
// least B * n_chunks entries (eloc_chunks); NULL selects the context's workspace.
gna_status run_eloc(gna_ctx* c, const double* theta, const int8_t* spins, int B, const double* base,
                    double* eloc, long long* nev, bool planes_ready = false, double* partial = nullptr,
                    int* cnt = nullptr, double* terms = nullptr) {
  {
    Timed tm(c, "k_zero_i64");
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, c->stream, nev, 1);
  }
  if (gna_status st = check_launch(c, "k_zero_i64")) return st;
  if (B == 0) return GNA_OK;
  int n_chunks = 1, ichunk = 1;
  eloc_chunks(c, B, &n_chunks, &ichunk);
  Net net = make_net(c, theta);
  const int items = B * n_chunks;
  if (!partial) partial = c->d_partial;
  if (!cnt) cnt = c->d_cnt;
  if (!terms) terms = c->d_terms;
  if (c->eloc_mode == GNA_ELOC_INCREMENTAL) {
    void* planes = c->d_inc_planes;
    double* lp_out = const_cast<double*>(base);   // the base pass also yields log psi(s)
    if (!planes_ready) {
      Timed tm(c, "k_inc_base");
      void* a1[] = {&net, &spins, &B, &planes, &lp_out};
      hipError_t e = hipLaunchKernel(c->ik.base, dim3(std::min(B, c->grid_inc_base)), dim3(64 * c->geo.wpc), a1,
                                     (size_t)c->geo.lds_bytes, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "k_inc_base");
    }
    IncNet inc = make_inc(c);
    if (c->pipe_el) {
      PipeGeo pg = c->pgeo_el;
      int grid_p = std::min(items, c->grid_pipe_el);
      if (grid_p < pg.xcd || grid_p % pg.xcd) pg.xcd = 1;   // small launches: plain order
      const uint2* sched = c->d_sched;
      const uint16_t* gtab = c->d_pipe_tab;
      {
        Timed tm(c, "k_eloc_pipe");
        void* a2[] = {&net, &inc, &pg, &sched, &gtab, &spins, &B, &planes, &n_chunks, &ichunk, &terms};
        hipError_t e = hipLaunchKernel(c->pk_el.eloc, dim3(grid_p), dim3(64 * pg.nw), a2, (size_t)pg.lds_bytes,
                                       c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "k_eloc_pipe");
      }
      if (gna_status st = check_launch(c, "k_eloc_pipe")) return st;
      {
        Timed tm(c, "k_eloc_terms");
        hipLaunchKernelGGL(k_eloc_terms, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, c->stream, spins, c->N,
                           c->d_edges, c->E, B, n_chunks, ichunk, terms, partial, cnt);
      }
      if (gna_status st = check_launch(c, "k_eloc_terms")) return st;
      Timed tm(c, "k_eloc_finalize");
      hipLaunchKernelGGL(k_eloc_finalize, dim3((B + 3) / 4), dim3(256), 0, c->stream, spins, c->N,
                         c->d_edges, c->E, c->jz, c->jxy, c->hb, c->cb, B, n_chunks, partial, cnt, eloc, nev);
      return check_launch(c, "k_eloc_finalize");
    }
    IncGeo ig = c->igeo;
    int grid_i = std::min(items, c->grid_inc);
    if (grid_i < ig.xcd || grid_i % ig.xcd) ig.xcd = 1;   // small launches: plain order
    {
      Timed tm(c, "k_eloc_inc");
      void* a2[] = {&net, &inc, &ig, &spins, &B, &planes, &n_chunks, &ichunk, &partial, &cnt};
      hipError_t e = hipLaunchKernel(c->ik.eloc, dim3(grid_i), dim3(64 * ig.nw), a2,
                                     (size_t)ig.lds_bytes, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "k_eloc_inc");
    }
    if (gna_status st = check_launch(c, "k_eloc_inc")) return st;
  } else {
    int grid = std::min(items, c->grid_eloc);
    void* args[] = {&net, &spins, &B, &base, &n_chunks, &ichunk, &partial, &cnt};
    if (gna_status st = launch(c, c->kern.eloc, grid, args, "k_eloc")) return st;
  }
  Timed tm(c, "k_eloc_finalize");
  hipLaunchKernelGGL(k_eloc_finalize, dim3((B + 3) / 4), dim3(256), 0, c->stream, spins, c->N,
                     c->d_edges, c->E, c->jz, c->jxy, c->hb, c->cb, B, n_chunks, partial, cnt, eloc, nev);
  return check_launch(c, "k_eloc_finalize");
}

gna_status run_vjp(gna_ctx* c, const double* theta, const int8_t* spins, int B, const double* cot, double* grad) {
  const int F = c->F, L = c->L, nW = c->tied ? 1 : L;
  const int rows = c->vjp_rows;
  {
    Timed tm(c, "k_fill");
    hipLaunchKernelGGL(k_fill, dim3((int)((rows * c->P + 255) / 256)), dim3(256), 0, c->stream, c->d_vjp_part, 0.0,
                       (int)(rows * c->P));
  }
  if (gna_status st = check_launch(c, "k_fill")) return st;
  if (B > 0) {
    {
      Timed tm(c, "k_prepare_vjp");
      c->vk.fk.prepare(theta, nW, c->act, c->d_vwfrag, c->d_vbias, c->d_vemb, c->stream);
      c->vk.prepare_bwd(theta, nW, c->d_wbwd, c->stream);
    }
    if (gna_status st = check_launch(c, "k_prepare_vjp")) return st;
    Net net = make_net(c, theta);
    net.wfrag = c->d_vwfrag;
    net.bias = c->d_vbias;
    net.emb = c->d_vemb;
    net.g = c->vgeo;
    VNet v{};
    v.n = c->N; v.F = F; v.L = L; v.tied = c->tied; v.dmax = c->dmax;
    v.act = c->act;
    v.npad = c->vgeo.npad; v.ntiles = c->vgeo.ntiles; v.wpc = c->vgeo.wpc;
    v.ell_idx = c->d_idx; v.ell_val = c->d_val; v.wbwd = c->d_wbwd; v.theta = theta;
    v.npar = (int)c->P;
    v.plane = (size_t)c->vgeo.npad * F;
    v.nplanes = c->nplanes;
    void* planes = c->d_planes;
    double* part = c->d_vjp_part;
    const int vthreads = 64 * c->vgeo.wpc;
    for (int b0 = 0; b0 < B; b0 += c->vjp_chunk) {
      int Bc = std::min(c->vjp_chunk, B - b0);
      int nplanes = c->nplanes;
      {
        Timed tm(c, "k_vjp_fwd");
        void* args[] = {&net, &spins, &b0, &Bc, &planes, &nplanes};
        hipError_t e = hipLaunchKernel(c->vk.fwd, dim3(std::min(Bc, c->vgrid_fwd)), dim3(vthreads), args,
                                       (size_t)c->vgeo.lds_bytes, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "k_vjp_fwd");
      }
      for (int layer = L - 1; layer >= 0; --layer) {
        {
          Timed tm(c, "k_vjp_dx");
          void* args[] = {&v, &layer, &b0, &Bc, &cot, &planes};
          hipError_t e = hipLaunchKernel(c->vk.dx, dim3(std::min(Bc, c->vgrid_dx)), dim3(vthreads), args,
                                         c->vdx_lds, c->stream);
          if (e != hipSuccess) return hip_fail(c, e, "k_vjp_dx");
        }
        {
          Timed tm(c, "k_vjp_dw");
          void* args[] = {&v, &layer, &Bc, &planes, &part};
          hipError_t e = hipLaunchKernel(c->vk.dw, dim3(rows), dim3(256), args, 0, c->stream);
          if (e != hipSuccess) return hip_fail(c, e, "k_vjp_dw");
        }
      }
      {
        Timed tm(c, "k_vjp_tail");
        void* args[] = {&v, &b0, &Bc, &spins, &cot, &planes, &part};
        hipError_t e = hipLaunchKernel(c->vk.tail, dim3(std::min(rows, Bc)), dim3(256), args, 0, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "k_vjp_tail");
      }
      if (gna_status st = check_launch(c, "k_vjp")) return st;
    }
  }
  Timed tm(c, "k_vjp_reduce");
  hipLaunchKernelGGL(k_vjp_reduce, dim3((int)((c->P + 63) / 64)), dim3(64), 0, c->stream, c->d_vjp_part, rows,
                     (int)c->P, grad);
  return check_launch(c, "k_vjp_reduce");
}

bool valid_ptr(const void* p) { return p != nullptr; }

// ---------------------------------------------------------------------------
// Shape of the incremental kernels: jobs in flight per workgroup (S), wave shape
// (8 waves of up to 4 tiles, or 16 waves of one tile) and samples in flight per
// XCD.  inc_configure derives the LDS layout, picks the instantiation and sizes
// the persistent grids; S < 0 asks for the largest S <= -S that fits.
// ---------------------------------------------------------------------------
struct IncShape {
  int S;        // 0: the layer-pipelined kernels (gna_pipe.h)
  bool wide;
  int per_xcd;
  int nw = 0;   // waves per workgroup; 0: as many as useful (8, or 16 when wide)
};

struct IncTune {
  IncShape el, sw;   // local-energy and sweep kernel shapes
};

std::mutex g_tune_mu;
std::vector<std::pair<std::string, IncTune>> g_tune;   // tuner cache (this process)

bool tune_lookup(const std::string& key, IncTune* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : g_tune)
    if (kv.first == key) {
      *out = kv.second;
      return true;
    }
  return false;
}

void tune_store(const std::string& key, const IncTune& v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : g_tune)
    if (kv.first == key) {
      kv.second = v;
      return;
    }
  g_tune.push_back({key, v});
}

// Tile schedule of the pipelined kernels: job slot j (setup at ticks = j mod D)
// runs layer l at tick j + extra + l (mod D).  Tile t (list positions 16t ..
// 16t+15) of a job holds registers from the first layer it computes or receives
// base rows for the next layer, to layer L.  Every (slot, tile) gets one (wave,
// register) pair whose live ticks it does not share, on the compute wave least
// loaded at those ticks.  A tick's two phases end at barriers, so what counts is
// the largest load of a wave in each phase: weighted, a tile's load at layer l is
// its message product (phase A; 16t below the product's rows) plus a share for
// base rows requested, and in phase B the gather, self product and activation
// (16t < |C_l|) plus the operand conversion (l < L) or the readout (l = L), or the
// conversion alone for a tile of base rows only; the heaviest tiles are placed
// first.  Unweighted, the load is the number of tiles with products, and tiles are
// placed in order of their first layer.  sched[tick mod D][wave] packs the
// (slot << 4 | tile) of registers 0..7 (0xff: none).  False when the tiles do not
// fit in maxt registers per wave.
bool pipe_schedule(const std::vector<int>& cmax, int L, int D, int extra, int nw, int sw, int maxt, bool weighted,
                   std::vector<uint2>* sched, int* max_load) {
  auto rows_at = [&](int l) { return std::max(l == 1 ? cmax[2] : cmax[l], cmax[l]); };   // products at layer l
  int top = 0;
  for (int l = 1; l <= L; ++l) top = std::max(top, rows_at(l));
  const int tmax = (top + 15) / 16;
  if (tmax > 16 || D > kPipeMaxD || maxt > kPipeMaxK) return false;
  std::vector<int> lf(tmax, L + 1);
  for (int t = 0; t < tmax; ++t)
    for (int l = L; l >= 1; --l)
      if (16 * t < rows_at(l) || (l < L && 16 * t < cmax[l + 1])) lf[t] = l;
  // weighted loads in tenths: phase A, phase B of tile t at layer l
  auto cost_a = [&](int t, int l) {
    int a = 16 * t < rows_at(l) ? 10 : 0;
    if (l < L && 16 * t < cmax[l + 1] && 16 * t + 16 > cmax[l]) a += 2;
    return weighted ? a : (16 * t < rows_at(l) ? 1 : 0);
  };
  auto cost_b = [&](int t, int l) {
    int b = 0;
    if (16 * t < cmax[l]) b = 10 + (l < L ? 3 : 6);
    else if (l < L && 16 * t < cmax[l + 1]) b = 3;
    return weighted ? b : 0;
  };
  struct Item { int j, t, w; };
  std::vector<Item> items;
  for (int t = 0; t < tmax; ++t)
    for (int j = 0; j < D; ++j)
      if (lf[t] <= L) {
        int wsum = 0;
        for (int l = lf[t]; l <= L; ++l) wsum += cost_b(t, l);
        items.push_back({j, t, wsum});
      }
  if (weighted)
    std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) { return a.w > b.w; });
  else
    std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) { return lf[a.t] < lf[b.t]; });
  std::vector<int> occ((size_t)D * nw * maxt, -1), la((size_t)D * nw, 0), lb((size_t)D * nw, 0);
  for (const Item& it : items) {
    int best_w = -1, best_k = -1;
    long long best_cost = 0;
    for (int w = 0; w < nw; ++w) {
      if (w == sw) continue;
      for (int k = 0; k < maxt; ++k) {
        bool free_ = true;
        int pa = 0, pb = 0, sum = 0;
        for (int l = lf[it.t]; l <= L && free_; ++l) {
          const int tau = (it.j + extra + l) % D;
          const size_t o = (size_t)tau * nw + w;
          if (occ[o * maxt + k] >= 0) free_ = false;
          const int ca = cost_a(it.t, l), cb = cost_b(it.t, l);
          if (ca + cb > 0) {
            pa = std::max(pa, la[o] + ca);
            pb = std::max(pb, lb[o] + cb);
            sum += la[o] + lb[o];
          }
        }
        if (!free_) continue;
        const long long cost = weighted ? ((long long)pb * 1000 + pa) * 100000 + (long long)sum * 10 + k
                                        : (long long)pa * 1000000 + sum * 100 + k;
        if (best_w < 0 || cost < best_cost) {
          best_w = w;
          best_k = k;
          best_cost = cost;
        }
        break;   // registers of one wave are interchangeable: the first free one
      }
    }
    if (best_w < 0) return false;
    for (int l = lf[it.t]; l <= L; ++l) {
      const int tau = (it.j + extra + l) % D;
      const size_t o = (size_t)tau * nw + best_w;
      occ[o * maxt + best_k] = it.j << 4 | it.t;
      la[o] += cost_a(it.t, l);
      lb[o] += cost_b(it.t, l);
    }
  }
  // bytes 6 and 7 of an entry: the waves with fewer phase-B tiles than the busiest
  // at that tick (the light waves, which take the tick's table conversion) and the
  // wave's rank among them (0xff: not light)
  if (maxt > 6) return false;
  sched->assign((size_t)kPipeMaxD * kMaxWaves, uint2{0xffffffffu, 0xffffffffu});
  int ml = 0;
  for (int tau = 0; tau < D; ++tau) {
    std::vector<int> nb(nw, 0);
    int nb_max = 0;
    for (int w = 0; w < nw; ++w) {
      if (w == sw) continue;
      unsigned long long v = ~0ULL;
      int busy = 0;
      for (int k = 0; k < maxt; ++k) {
        const int o = occ[((size_t)tau * nw + w) * maxt + k];
        if (o >= 0) {
          v = (v & ~(0xffULL << (8 * k))) | ((unsigned long long)o << (8 * k));
          const int l = ((tau - (o >> 4) - extra) % D + D) % D;
          if (l >= 1 && 16 * (o & 15) < rows_at(l)) ++busy;
          if (l >= 1 && 16 * (o & 15) < cmax[l]) ++nb[w];
        }
      }
      (*sched)[(size_t)tau * kMaxWaves + w] = uint2{(unsigned)v, (unsigned)(v >> 32)};
      ml = std::max(ml, busy);
      nb_max = std::max(nb_max, nb[w]);
    }
    int nlight = 0;
    for (int w = 0; w < nw; ++w)
      if (w != sw && nb[w] < nb_max) ++nlight;
    for (int w = 0, rank = 0; w < nw; ++w) {
      if (w == sw) continue;
      const bool light = nlight == 0 || nb[w] < nb_max;   // all compute waves when equal
      unsigned& hi = (*sched)[(size_t)tau * kMaxWaves + w].y;
      hi = (hi & 0xffffu) | (unsigned)(nlight == 0 ? nw - 1 : nlight) << 16 | (unsigned)(light ? rank++ : 0xff) << 24;
    }
  }
  if (max_load) *max_load = ml;
  return true;
}

// Shape of a pipelined kernel (which: 1 local energy, 2 sweep): pools, LDS layout,
// tile schedule, instantiation and persistent grid.
gna_status pipe_configure(gna_ctx* c, IncShape shp, int which) {
  if (!c->pipe_ok) return fail(c, GNA_UNSUPPORTED, "pipelined kernels: the graph's balls exceed their tables");
  if (c->act != 0) return fail(c, GNA_UNSUPPORTED, "pipelined kernels: tanh only (ReLU + layer normalisation runs grouped)");
  const int F = c->F, L = c->L, N = c->N, dmax = c->dmax;
  const int nt = shp.wide ? 1024 : 512;
  const PipeKern pk = pipe_pick(c->prec, F, nt);
  if (!pk.eloc) return fail(c, GNA_UNSUPPORTED, "pipelined kernels: no instantiation for this precision");
  PipeGeo g{};
  g.nw = nt / 64;
  g.sw = g.nw - 1;
  g.extra = 1;
  g.D = L + 1 + g.extra;
  if (g.D > kPipeMaxD) return fail(c, GNA_UNSUPPORTED, "pipelined kernels: too many layers");
  g.row_elems = (int)((F * c->sz_Acc + kRowPadBytes) / c->sz_Acc);
  int rows = 0;
  for (int pi = 0; pi < kPipeMaxL; ++pi) {
    g.pool_cnt[pi] = 1;
    g.pool_rows[pi] = 0;
    g.pool_base[pi] = 0;
  }
  for (int pi = 0; pi < L; ++pi) {
    g.pool_cnt[pi] = L - pi;
    g.pool_rows[pi] = pi == 0 ? c->ball_cmax[2] : c->ball_ringmax[pi + 2];
    g.pool_base[pi] = rows;
    rows += g.pool_cnt[pi] * g.pool_rows[pi];
  }
  if (rows > 65535) return fail(c, GNA_UNSUPPORTED, "pipelined kernels: LDS rows exceed 16-bit indices");
  g.tabw = c->pipe_tabw;
  g.r8 = c->inc_r8;
  g.ntab = L + 1;
  g.spw = (int)((c->geo.npad + 15) / 16 * 16);
  g.xcd = 8;   // MI355X: 8 XCDs, workgroups assigned round-robin
  size_t o = 0;
  auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
  g.off_w = (int)o; o = al(o + c->inc_w_bytes);
  g.off_arena = (int)o; o = al(o + (size_t)rows * g.row_elems * c->sz_Acc);
  g.off_tab = (int)o; o = al(o + (size_t)g.ntab * g.tabw * 2);
  g.off_sp = (int)o; o = al(o + (size_t)(g.D + 1) * g.spw);
  g.off_red = (int)o; o = al(o + (size_t)4 * kMaxWaves * 8);
  g.off_bias = (int)o; o = al(o + (size_t)F * c->sz_Acc);
  g.off_emb = (int)o; o = al(o + (size_t)2 * F * c->sz_Acc);
  g.off_head = (int)o; o = al(o + (size_t)2 * (F + 3) * 8);
  g.off_ev = (int)o; o = al(o + (size_t)N * dmax * c->sz_Acc);
  g.off_edges = (int)o; o = al(o + (size_t)std::max(c->E, 1) * 4);
  g.rows_max = 1;   // ring rows copied in one tick: rings 3 .. L+1, one job at each layer
  for (int sr = 3; sr <= L + 1; ++sr) g.rows_max += c->ball_ringmax[sr];
  g.off_rows = (int)o; o = al(o + (size_t)2 * g.rows_max * 8);
  g.lds_bytes = (int)o;
  // the row list holds source offsets in 16-byte vectors of the planes as 32-bit words
  if ((double)c->max_batch * 2 * L * c->geo.npad * F * c->sz_Acc / 16 >= 4294967296.0)
    return fail(c, GNA_UNSUPPORTED, "pipelined kernels: the planes exceed 32-bit vector offsets");
  if (o + sizeof(PipeState) + 256 > c->lds_max)
    return fail(c, GNA_UNSUPPORTED, "pipelined kernels: the shape does not fit in LDS");
  std::vector<uint2> sched;
  int ml = 0;
  if (!pipe_schedule(c->ball_cmax, L, g.D, g.extra, g.nw, g.sw, pk.maxt, true, &sched, &ml) &&
      !pipe_schedule(c->ball_cmax, L, g.D, g.extra, g.nw, g.sw, pk.maxt, false, &sched, &ml))
    return fail(c, GNA_UNSUPPORTED, "pipelined kernels: the tiles do not fit in the wave registers");
  const void* fn = which == 1 ? pk.eloc : pk.sweep;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, g.lds_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, GNA_HIP_ERROR, "hipFuncSetAttribute: the pipelined kernel's LDS size was not accepted");
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, nt, g.lds_bytes) != hipSuccess || nb < 1) nb = 1;
  (void)hipGetLastError();
  uint2* dst = c->d_sched + (size_t)(which == 1 ? 0 : 1) * kPipeMaxD * kMaxWaves;
  if (hipMemcpy(dst, sched.data(), sched.size() * sizeof(uint2), hipMemcpyHostToDevice) != hipSuccess)
    return fail(c, GNA_HIP_ERROR, "hipMemcpy: pipelined tile schedule");
  if (which == 1) {
    c->pgeo_el = g;
    c->pk_el = pk;
    c->grid_pipe_el = c->n_cu * nb;
  } else {
    c->pgeo_sw = g;
    c->pk_sw = pk;
    c->grid_pipe_sw = c->n_cu * nb;
  }
  return GNA_OK;
}

// which: 1 the local-energy kernel, 2 the sweep kernel, 3 both
gna_status inc_configure(gna_ctx* c, IncShape shp, int which) {
  const int F = c->F, N = c->N, dmax = c->dmax;
  const int max_rows = c->inc_max_rows, max_ball = c->inc_max_ball, max_tiles = c->inc_max_tiles;
  IncGeo base{};
  base.xcd = 8;   // MI355X: 8 XCDs, workgroups assigned round-robin
  base.rows = max_rows;
  base.tabw = (c->inc_r8 + max_ball * dmax + 7) / 8 * 8;
  base.row_elems = (int)((4 * (F / 4) * c->sz_Acc + kRowPadBytes) / c->sz_Acc);
  const int chunk_cap = 64 * kMaxWaves / 2;   // bonds per work item: at most one per thread
  auto geometry = [&](int S, bool wide, int nw_req, IncGeo* out, int* maxt) {
    const int tiles = S * max_tiles;
    const int nw = std::min(nw_req > 0 ? nw_req : (wide ? kMaxWaves : kMaxWaves / 2), tiles);
    const int mt = (tiles + nw - 1) / nw;   // tiles per wave
    if (mt > (wide ? 1 : 4)) return false;
    size_t o = 0;
    auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
    IncGeo t = base;
    t.S = S;
    t.nw = nw;
    t.off_w = (int)o; o = al(o + c->inc_w_bytes);
    t.off_buf = (int)o; o = al(o + (size_t)S * max_rows * base.row_elems * c->sz_Acc);
    t.off_tab = (int)o; o = al(o + (size_t)S * base.tabw * 2);
    t.spw = (int)al(c->geo.npad);
    t.off_sp = (int)o; o = al(o + (size_t)S * t.spw);
    t.off_red = (int)o; o = al(o + (size_t)kIncMaxSwaps * 2 * kMaxWaves * 8);
    t.off_bias = (int)o; o = al(o + (size_t)F * c->sz_Acc);
    t.off_emb = (int)o; o = al(o + (size_t)2 * F * c->sz_Acc);
    t.off_head = (int)o; o = al(o + (size_t)2 * (F + 3) * 8);
    t.off_ev = (int)o; o = al(o + (size_t)N * dmax * c->sz_Acc);
    t.off_list = (int)o; o = al(o + (size_t)chunk_cap * 4);
    t.off_cpy = (int)o; o = al(o + (size_t)S * max_rows * 16);
    // the sweep keeps the bond list in LDS for its proposal draws when it fits
    t.off_edges = -1;
    const size_t eb = al((size_t)std::max(c->E, 1) * 8);
    if ((which & 2) && o + eb + 2048 <= c->lds_max) {
      t.off_edges = (int)o;
      o += eb;
    }
    t.lds_bytes = (int)o;
    if (o + 2048 > c->lds_max) return false;   // static LDS of the kernels
    *out = t;
    *maxt = mt;
    return true;
  };
  if (shp.S == 0) {   // the layer-pipelined kernels
    for (int w = 1; w <= 2; ++w) {
      if (!(which & w)) continue;
      if (gna_status st = pipe_configure(c, shp, w)) return st;
      if (w == 1) {
        c->pipe_el = true;
        c->inc_wide = shp.wide;
        c->inc_maxt = c->pk_el.maxt;
        c->inc_per_xcd = std::max(1, shp.per_xcd);
        c->inc_chunk_cap = std::min(chunk_cap, kPipeMaskWords * 32);
        c->grid_inc = c->grid_pipe_el;
      } else {
        c->pipe_sw = true;
        c->inc_sw_wide = shp.wide;
        c->inc_sw_maxt = c->pk_sw.maxt;
      }
    }
    return GNA_OK;
  }
  IncGeo ig{};
  int maxt = 0;
  if (shp.S < 0) {
    for (int S = std::min(-shp.S, kIncMaxSwaps); S >= 1 && !maxt; --S)
      if (geometry(S, shp.wide, shp.nw, &ig, &maxt)) shp.S = S;
  } else if (shp.S >= 1 && shp.S <= kIncMaxSwaps) {
    geometry(shp.S, shp.wide, shp.nw, &ig, &maxt);
  }
  if (maxt == 0)
    return fail(c, GNA_UNSUPPORTED, "incremental kernel shape does not fit (LDS, or more than 4 tiles per wave)");
  const int tpw = c->tpw, nch = c->nch;
  IncKern ik;
  switch (c->prec) {
    case GNA_FP64: ik = inc_pick_f<PF64>(F, tpw, nch, maxt, shp.wide); break;
    case GNA_FP32: ik = inc_pick_f<PF32>(F, tpw, nch, maxt, shp.wide); break;
    case GNA_BF16_1X:
      if (F == 16) ik = inc_pick<PBF161, 16>(tpw, nch, maxt, shp.wide);
      else if (F == 32) ik = inc_pick<PBF16W1, 32>(tpw, nch, maxt, shp.wide);
      else ik = inc_pick<PBF16W1, 64>(tpw, nch, maxt, shp.wide);
      break;
    default:
      if (c->split_w) ik = F == 32 ? inc_pick<PBF16S<32>, 32>(tpw, nch, maxt, shp.wide)
                                   : inc_pick<PBF16S<64>, 64>(tpw, nch, maxt, shp.wide);
      else if (F == 16) ik = inc_pick<PBF16, 16>(tpw, nch, maxt, shp.wide);
      else if (F == 32) ik = inc_pick<PBF16W, 32>(tpw, nch, maxt, shp.wide);
      else ik = inc_pick<PBF16W, 64>(tpw, nch, maxt, shp.wide);
  }
  bool attr_fail = false;
  auto occ2 = [&](const void* fn, int threads_, int lds) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) attr_fail = true;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads_, lds) != hipSuccess || nb < 1) nb = 1;
    (void)hipGetLastError();
    return nb;
  };
  const int g_base = c->n_cu * occ2(ik.base, 64 * c->geo.wpc, c->geo.lds_bytes);
  const int g_el = (which & 1) ? c->n_cu * occ2(ik.eloc, 64 * ig.nw, ig.lds_bytes) : 0;
  const int g_sw = (which & 2) ? c->n_cu * occ2(ik.sweep, 64 * ig.nw, ig.lds_bytes) : 0;
  if (attr_fail)
    return fail(c, GNA_HIP_ERROR, "hipFuncSetAttribute: the incremental kernels' LDS size was not accepted");
  c->ik.base = ik.base;   // the base pass does not depend on the shape
  c->grid_inc_base = g_base;
  if (which & 1) {
    c->pipe_el = false;
    c->igeo = ig;
    c->ik.eloc = ik.eloc;
    c->inc_wide = shp.wide;
    c->inc_maxt = maxt;
    c->inc_per_xcd = std::max(1, shp.per_xcd);
    c->inc_chunk_cap = std::min(chunk_cap, 64 * ig.nw);
    c->grid_inc = g_el;
  }
  if (which & 2) {
    c->pipe_sw = false;
    c->igeo_sw = ig;
    c->ik.sweep = ik.sweep;
    c->inc_sw_wide = shp.wide;
    c->inc_sw_maxt = maxt;
    c->grid_sweep_inc = g_sw;
  }
  return GNA_OK;
}

// the shapes in use (for restoring them after a failed change)
IncShape shape_el(const gna_ctx* c) {
  if (c->pipe_el) return IncShape{0, c->inc_wide, c->inc_per_xcd, 0};
  return IncShape{c->igeo.S, c->inc_wide, c->inc_per_xcd, c->igeo.nw};
}
IncShape shape_sw(const gna_ctx* c) {
  if (c->pipe_sw) return IncShape{0, c->inc_sw_wide, 1, 0};
  return IncShape{c->igeo_sw.S, c->inc_sw_wide, 1, c->igeo_sw.nw};
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

gna_status gna_init(const gna_config* cfg, gna_ctx** out) {
  auto init_fail = [&](gna_status st, const std::string& m) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    g_init_err = m;
    return st;
  };
  if (!out) return init_fail(GNA_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return init_fail(GNA_INVALID_ARG, "cfg is NULL");
  const int N = cfg->n_sites, E = cfg->n_edges, F = cfg->n_features, L = cfg->n_layers;
  if (N < 2 || N > 4096) return init_fail(GNA_INVALID_ARG, "n_sites must be in [2, 4096]");
  if (E < 0) return init_fail(GNA_INVALID_ARG, "n_edges must be >= 0");
  if (E > 0 && !cfg->edges) return init_fail(GNA_INVALID_ARG, "edges is NULL");
  if (F != 16 && F != 32 && F != 64) return init_fail(GNA_UNSUPPORTED, "n_features must be 16, 32 or 64");
  if (L < 0 || L > 16) return init_fail(GNA_UNSUPPORTED, "n_layers must be in [0, 16]");
  if (cfg->tied != 0 && cfg->tied != 1) return init_fail(GNA_INVALID_ARG, "tied must be 0 or 1");
  if (cfg->precision < GNA_FP64 || cfg->precision > GNA_BF16_1X) return init_fail(GNA_INVALID_ARG, "unknown precision");
  if (cfg->eloc_mode != GNA_ELOC_FULL && cfg->eloc_mode != GNA_ELOC_INCREMENTAL)
    return init_fail(GNA_INVALID_ARG, "unknown eloc_mode");
  if (cfg->activation != GNA_ACT_TANH && cfg->activation != GNA_ACT_RELU_LN)
    return init_fail(GNA_INVALID_ARG, "unknown activation");
  if (cfg->reserved != 0) return init_fail(GNA_INVALID_ARG, "reserved must be 0");
  // Six normalised layers carry the 8-bit rounding of bfloat16 weights to the
  // output at unit scale (about 0.1 per site at 432 sites, L = 6, F = 64), far
  // outside the BF16 accuracy bound of 1e-3 per site: under this activation GNA_BF16
  // carries each weight as a hi + lo pair of bfloat16 values (F a multiple of 32),
  // and single-pass BF16, whose operands are single bfloat16 values by definition,
  // is refused.
  if (cfg->activation == GNA_ACT_RELU_LN && cfg->precision == GNA_BF16_1X)
    return init_fail(GNA_UNSUPPORTED, "ReLU + layer normalisation needs split (hi + lo) bfloat16 layer products "
                                      "(single bfloat16 weights miss the BF16 accuracy bound)");
  if (cfg->activation == GNA_ACT_RELU_LN && cfg->precision == GNA_BF16 && F % 32 != 0)
    return init_fail(GNA_UNSUPPORTED, "ReLU + layer normalisation in BF16 needs n_features a multiple of 32 "
                                      "(split bfloat16 weights)");
  if (cfg->eloc_mode == GNA_ELOC_INCREMENTAL && !cfg->tied)
    return init_fail(GNA_UNSUPPORTED, "incremental local energy needs tied weights");
  if (cfg->eloc_mode == GNA_ELOC_INCREMENTAL && L < 1)
    return init_fail(GNA_UNSUPPORTED, "incremental local energy needs n_layers >= 1");
  if (cfg->max_batch < 0) return init_fail(GNA_INVALID_ARG, "max_batch must be >= 0");
  if (cfg->act_budget_bytes < 0) return init_fail(GNA_INVALID_ARG, "act_budget_bytes must be >= 0");
  if (!std::isfinite(cfg->jz) || !std::isfinite(cfg->jxy)) return init_fail(GNA_INVALID_ARG, "couplings must be finite");
  // graph validation (host, before any device call)
  std::vector<int> deg(N, 0);
  std::set<std::pair<int, int>> seen;
  for (int e = 0; e < E; ++e) {
    int a = cfg->edges[2 * e], b = cfg->edges[2 * e + 1];
    if (a < 0 || a >= N || b < 0 || b >= N)
      return init_fail(GNA_BAD_GRAPH, "edge " + std::to_string(e) + " has an endpoint out of range");
    if (a == b) return init_fail(GNA_BAD_GRAPH, "edge " + std::to_string(e) + " is a self-loop");
    if (!seen.insert({std::min(a, b), std::max(a, b)}).second)
      return init_fail(GNA_BAD_GRAPH, "edge " + std::to_string(e) + " repeats a bond");
    ++deg[a];
    ++deg[b];
  }
  int dmax = 1;
  for (int d : deg) dmax = std::max(dmax, d);
  dmax = (dmax + 3) / 4 * 4;   // the gather loop reads neighbours four at a time

  gna_ctx* c = new gna_ctx();
  c->N = N; c->E = E; c->F = F; c->L = L; c->tied = cfg->tied; c->prec = cfg->precision;
  c->act = cfg->activation;
  c->jz = cfg->jz; c->jxy = cfg->jxy; c->max_batch = cfg->max_batch;
  c->stream = reinterpret_cast<hipStream_t>(cfg->stream);
  c->P = param_count(F, L, cfg->tied);
  c->dmax = dmax;
  // split BF16 under ReLU + layer normalisation: weights as hi + lo bfloat16 pairs
  c->split_w = c->prec == GNA_BF16 && c->act == GNA_ACT_RELU_LN;
  c->sz_W = (c->prec == GNA_FP64) ? 8 : (c->prec == GNA_FP32 || c->split_w ? 4 : 2);
  c->sz_Acc = (c->prec == GNA_FP64) ? 8 : 4;

  auto bail = [&](gna_status st, const std::string& m) {
    const std::string msg = m;   // m may be c->err
    free_all(c);
    delete c;
    return init_fail(st, msg);
  };
  hipError_t he = hipGetDevice(&c->device);
  if (he != hipSuccess) return bail(GNA_HIP_ERROR, std::string("hipGetDevice: ") + hipGetErrorString(he));
  hipDeviceProp_t prop;
  he = hipGetDeviceProperties(&prop, c->device);
  if (he != hipSuccess) return bail(GNA_HIP_ERROR, std::string("hipGetDeviceProperties: ") + hipGetErrorString(he));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return bail(GNA_UNSUPPORTED, std::string("built for gfx950, device is ") + prop.gcnArchName);
  c->n_cu = prop.multiProcessorCount;
  const size_t lds_max = prop.sharedMemPerBlock;
  {
    // the static scratch of gna_local_energy_noalloc on this device (the current one)
    const hipError_t se = static_scratch(c->device, &c->scratch_dev);
    if (se != hipSuccess) c->scratch_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(se);
  }

  // ---- geometry: tiles per wave, waves per workgroup, gather chunks, buffers
  Geo& g = c->geo;
  g.ntiles = (N + 15) / 16;
  g.npad = 16 * g.ntiles;
  const char* env_tpw = std::getenv("GNA_TILES_PER_WAVE");
  int tpw = 0;
  if (env_tpw) tpw = std::atoi(env_tpw);
  // the evaluator kernels are built for at most 8 waves (256 VGPRs per lane)
  auto max_waves = [](int) { return kMaxWaves / 2; };
  if (tpw != 1 && tpw != 2 && tpw != 4) {
    tpw = 1;
    while (tpw < 4 && (g.ntiles + tpw - 1) / tpw > max_waves(tpw)) tpw *= 2;
  }
  g.wpc = (g.ntiles + tpw - 1) / tpw;
  if (g.wpc > max_waves(tpw)) return bail(GNA_UNSUPPORTED, "n_sites too large for one workgroup (max 512)");
  // every wave owns exactly tpw tiles: padding nodes (zero adjacency, left out of the
  // readout) fill the last ones, so the kernels need no per-tile branches
  g.ntiles = g.wpc * tpw;
  g.npad = 16 * g.ntiles;
  c->tpw = tpw;
  const size_t w_bytes = (size_t)2 * F * F * c->sz_W;
  auto layout = [&](int nch, int nbuf) -> size_t {
    const int cs = (F / 4) / nch;
    g.nbuf = nbuf;
    g.row_elems = (int)((4 * cs * c->sz_Acc + kRowPadBytes) / c->sz_Acc);
    g.buf_elems = g.npad * g.row_elems;
    size_t o = 0;
    auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
    g.off_w = (int)o; o = al(o + w_bytes);
    g.off_h = (int)o; o = al(o + (size_t)nbuf * g.buf_elems * c->sz_Acc);
    g.off_sp = (int)o; o = al(o + g.npad);
    g.off_idx = (int)o; o = al(o + (size_t)g.npad * dmax * 4);
    g.off_val = (int)o; o = al(o + (size_t)g.npad * dmax * c->sz_Acc);
    g.off_red = (int)o; o = al(o + kRedSlots * 8);
    g.off_bias = (int)o; o = al(o + (size_t)(cfg->tied ? 1 : std::max(L, 1)) * F * c->sz_Acc);
    g.off_emb = (int)o; o = al(o + (size_t)2 * F * c->sz_Acc);
    g.off_head = (int)o; o = al(o + (size_t)2 * (F + 3) * 8);
    g.lds_bytes = (int)o;
    return o + 64;  // static shared scalars
  };
  int nch = 0;
  const int cand[4][2] = {{1, 2}, {1, 1}, {4, 2}, {4, 1}};
  for (auto& cd : cand) {
    if ((F / 16) % cd[0] != 0) continue;   // message chunks split the output 16-feature tiles
    if (layout(cd[0], cd[1]) <= lds_max) { nch = cd[0]; break; }
  }
  if (!nch) return bail(GNA_UNSUPPORTED, "configuration does not fit in LDS");
  c->nch = nch;
  switch (c->prec) {
    case GNA_FP64: c->kern = pick_f<PF64>(F, tpw, nch); break;
    case GNA_FP32: c->kern = pick_f<PF32>(F, tpw, nch); break;
    case GNA_BF16_1X:
      c->kern = (F == 16) ? pick_nch<PBF161, 16>(tpw, nch)
                          : (F == 32 ? pick_nch<PBF16W1, 32>(tpw, nch) : pick_nch<PBF16W1, 64>(tpw, nch));
      break;
    default:
      // bf16: the K=32 instruction where F allows, the K=16 one at F = 16; split
      // weights under ReLU + layer normalisation (F >= 32)
      if (c->split_w)
        c->kern = F == 32 ? pick_nch<PBF16S<32>, 32>(tpw, nch) : pick_nch<PBF16S<64>, 64>(tpw, nch);
      else
        c->kern = (F == 16) ? pick_nch<PBF16, 16>(tpw, nch)
                            : (F == 32 ? pick_nch<PBF16W, 32>(tpw, nch) : pick_nch<PBF16W, 64>(tpw, nch));
      break;
  }
  const int threads = 64 * g.wpc;
  bool attr_fail = false;
  auto occ = [&](const void* fn) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, g.lds_bytes) != hipSuccess)
      attr_fail = true;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, g.lds_bytes) != hipSuccess || nb < 1) nb = 1;
    (void)hipGetLastError();
    return nb;
  };
  c->grid_logpsi = c->n_cu * occ(c->kern.logpsi);
  c->grid_eloc = c->n_cu * occ(c->kern.eloc);
  c->grid_sweep = c->n_cu * occ(c->kern.sweep);
  c->max_chunks = std::max(1, (E + 7) / 8);
  if (attr_fail) return bail(GNA_HIP_ERROR, "hipFuncSetAttribute: the evaluator's LDS size was not accepted");

  // ---- host graph tables: ELL (padding points at the node itself with value 0)
  std::vector<int> idx((size_t)g.npad * dmax);
  std::vector<double> val((size_t)g.npad * dmax, 0.0);
  std::vector<int> fill(g.npad, 0);
  for (int n = 0; n < g.npad; ++n)
    for (int d = 0; d < dmax; ++d) idx[(size_t)n * dmax + d] = n;
  std::vector<int> hedges(2 * (size_t)std::max(E, 1), 0);
  for (int e = 0; e < E; ++e) {
    const int a = cfg->edges[2 * e], b = cfg->edges[2 * e + 1];
    hedges[2 * e] = a;
    hedges[2 * e + 1] = b;
    const double w = 1.0 / std::sqrt((double)deg[a] * (double)deg[b]);
    idx[(size_t)a * dmax + fill[a]] = b; val[(size_t)a * dmax + fill[a]] = w; ++fill[a];
    idx[(size_t)b * dmax + fill[b]] = a; val[(size_t)b * dmax + fill[b]] = w; ++fill[b];
  }
  std::vector<float> val32(val.begin(), val.end());

  gna_status st = GNA_OK;
  const size_t MB = (size_t)std::max(1, c->max_batch);
  if ((st = dev_alloc(c, &c->d_edges, hedges.size() * 4)) ||
      (st = dev_alloc(c, &c->d_idx, idx.size() * 4)) ||
      (st = dev_alloc(c, &c->d_val64, val.size() * 8)) ||
      (st = dev_alloc(c, &c->d_val, val.size() * c->sz_Acc)) ||
      (st = dev_alloc(c, &c->d_wfrag, (size_t)(c->tied ? 1 : L) * w_bytes)) ||
      (st = dev_alloc(c, &c->d_bias, (size_t)(c->tied ? 1 : std::max(L, 1)) * F * c->sz_Acc)) ||
      (st = dev_alloc(c, &c->d_emb, (size_t)2 * F * c->sz_Acc)) ||
      (st = dev_alloc(c, &c->d_base, MB * 2 * 8)) ||
      (st = dev_alloc(c, &c->d_partial, MB * c->max_chunks * 4 * 8)) ||
      (st = dev_alloc(c, &c->d_cnt, MB * c->max_chunks * 4)) ||
      (st = dev_alloc(c, &c->d_nev, 8)) ||
      (st = dev_alloc(c, &c->d_cot, MB * 2 * 8)) ||
      (st = dev_alloc(c, &c->d_eloc, MB * 2 * 8)))
    return bail(st, c->err);
  // duplicate grouping: hash table of at least twice the batch, four int rows
  c->grp_T = 1;
  while ((size_t)c->grp_T < 2 * MB) c->grp_T *= 2;
  if ((st = dev_alloc(c, &c->d_grp_key, (size_t)c->grp_T * 8)) ||
      (st = dev_alloc(c, &c->d_grp_val, (size_t)c->grp_T * 4)) ||
      (st = dev_alloc(c, &c->d_grp_row, 4 * MB * 4)))
    return bail(st, c->err);
  // reverse pass: FP64 for FP64, FP32 otherwise; its own geometry and weights
  {
    const bool v64 = (c->prec == GNA_FP64);
    const size_t vw_bytes = (size_t)2 * F * F * (v64 ? 8 : 4);
    Geo saved = g;
    int vnch = 0;
    size_t wb_save = 0;
    (void)wb_save;
    // same tile split as the forward; pick chunks / buffers for the FP32/FP64 operands
    auto vlayout = [&](int nch_, int nbuf) -> size_t {
      const int cs = (F / 4) / nch_;
      Geo& h = c->vgeo;
      h = saved;
      h.nbuf = nbuf;
      h.row_elems = (int)((4 * cs * c->sz_Acc + kRowPadBytes) / c->sz_Acc);
      h.buf_elems = h.npad * h.row_elems;
      size_t o = 0;
      auto al = [](size_t x) { return (x + 15) & ~(size_t)15; };
      h.off_w = (int)o; o = al(o + vw_bytes);
      h.off_h = (int)o; o = al(o + (size_t)nbuf * h.buf_elems * c->sz_Acc);
      h.off_sp = (int)o; o = al(o + h.npad);
      h.off_idx = (int)o; o = al(o + (size_t)h.npad * dmax * 4);
      h.off_val = (int)o; o = al(o + (size_t)h.npad * dmax * c->sz_Acc);
      h.off_red = (int)o; o = al(o + kRedSlots * 8);
      h.off_bias = (int)o; o = al(o + (size_t)(cfg->tied ? 1 : std::max(L, 1)) * F * c->sz_Acc);
      h.off_emb = (int)o; o = al(o + (size_t)2 * F * c->sz_Acc);
      h.off_head = (int)o; o = al(o + (size_t)2 * (F + 3) * 8);
      h.lds_bytes = (int)o;
      return o + 64;
    };
    for (auto& cd : cand) {
      if ((F / 16) % cd[0] != 0) continue;
      if (vlayout(cd[0], cd[1]) <= lds_max) { vnch = cd[0]; break; }
    }
    if (!vnch) return bail(GNA_UNSUPPORTED, "reverse pass does not fit in LDS");
    c->vk = v64 ? vpick_f<PF64>(F, tpw, vnch) : vpick_f<PF32>(F, tpw, vnch);
    const int vthreads = 64 * c->vgeo.wpc;
    auto vocc = [&](const void* fn, int lds) {
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) attr_fail = true;
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, vthreads, lds) != hipSuccess || nb < 1) nb = 1;
      (void)hipGetLastError();
      return nb;
    };
    c->vgrid_fwd = c->n_cu * vocc(c->vk.fwd, c->vgeo.lds_bytes);
    // within the forward layout's LDS, which holds the same fragments and adjacency
    c->vdx_lds = vw_bytes + (size_t)c->vgeo.npad * dmax * ((v64 ? 8 : 4) + 4);
    c->vgrid_dx = c->n_cu * vocc(c->vk.dx, (int)c->vdx_lds);
    if (attr_fail) return bail(GNA_HIP_ERROR, "hipFuncSetAttribute: the reverse pass's LDS size was not accepted");
    c->vjp_rows = 3 * c->n_cu;   // three 4-wave workgroups of k_vjp_dw per CU (164 registers per lane)
    c->nplanes = 2 * L + 5 + (c->act ? L : 0);   // + post-ReLU rows Y^1..Y^L
    const int64_t per_sample = (int64_t)c->nplanes * c->vgeo.npad * F * (int64_t)c->sz_Acc;
    const int64_t budget = cfg->act_budget_bytes ? cfg->act_budget_bytes : ((int64_t)16 << 30);
    int64_t chunk = std::max<int64_t>(1, budget / std::max<int64_t>(per_sample, 1));
    chunk = std::min<int64_t>(chunk, (int64_t)MB);
    c->vjp_chunk = (int)chunk;
    if ((st = dev_alloc(c, &c->d_vwfrag, (size_t)(c->tied ? 1 : std::max(L, 1)) * vw_bytes)) ||
        (st = dev_alloc(c, &c->d_vbias, (size_t)(c->tied ? 1 : std::max(L, 1)) * F * c->sz_Acc)) ||
        (st = dev_alloc(c, &c->d_vemb, (size_t)2 * F * c->sz_Acc)) ||
        (st = dev_alloc(c, &c->d_wbwd, (size_t)(c->tied ? 1 : std::max(L, 1)) * vw_bytes)) ||
        (st = dev_alloc(c, &c->d_planes, (size_t)chunk * per_sample)) ||
        (st = dev_alloc(c, &c->d_vjp_part, (size_t)c->vjp_rows * c->P * 8)))
      return bail(st, c->err);
  }
  // incremental local energy: per-bond nested balls, base planes, kernels
  c->eloc_mode = cfg->eloc_mode;
  if (c->eloc_mode == GNA_ELOC_INCREMENTAL) {
    std::vector<std::vector<int>> adj(N);
    for (int e = 0; e < E; ++e) {
      adj[cfg->edges[2 * e]].push_back(cfg->edges[2 * e + 1]);
      adj[cfg->edges[2 * e + 1]].push_back(cfg->edges[2 * e]);
    }
    // node list of bond e: C_0 = {i, j}, then the nodes at distance 1, 2, ..., L+1
    // (each ring sorted), so that C_l is a prefix
    std::vector<std::vector<int>> lists(std::max(E, 1));
    std::vector<int> cnt((size_t)std::max(E, 1) * (L + 2), 0);
    int max_rows = 2, max_ball = 2;
    {
      std::vector<int> mark(N, 0);
      for (int e = 0; e < E; ++e) {
        std::vector<int>& lst = lists[e];
        const int a = cfg->edges[2 * e], bb = cfg->edges[2 * e + 1];
        lst = {std::min(a, bb), std::max(a, bb)};
        for (int u : lst) mark[u] = 1;
        cnt[(size_t)e * (L + 2)] = 2;
        size_t r0 = 0;
        for (int l = 1; l <= L + 1; ++l) {
          const size_t r1 = lst.size();
          std::vector<int> ring;
          for (size_t r = r0; r < r1; ++r)
            for (int v : adj[lst[r]])
              if (!mark[v]) { mark[v] = 1; ring.push_back(v); }
          std::sort(ring.begin(), ring.end());
          lst.insert(lst.end(), ring.begin(), ring.end());
          cnt[(size_t)e * (L + 2) + l] = (int)lst.size();
          r0 = r1;
        }
        for (int u : lst) mark[u] = 0;
        max_rows = std::max(max_rows, (int)lst.size());
        max_ball = std::max(max_ball, cnt[(size_t)e * (L + 2) + L]);
      }
    }
    const int r8 = (max_rows + 7) / 8 * 8;
    const int max_tiles = (max_ball + 15) / 16;
    // per bond: r8 node slots, then |C_L| x dmax neighbour list positions (16-bit
    // entries: N <= 4096), padded to whole 16-byte vectors
    std::vector<int2> meta(std::max(E, 1), int2{0, 0});
    std::vector<uint16_t> tabv;
    {
      std::vector<int> pos(N, -1);
      for (int e = 0; e < E; ++e) {
        const std::vector<int>& lst = lists[e];
        meta[e].x = (int)tabv.size();
        for (int r = 0; r < r8; ++r) tabv.push_back(r < (int)lst.size() ? (uint16_t)lst[r] : (uint16_t)0xffff);
        for (size_t r = 0; r < lst.size(); ++r) pos[lst[r]] = (int)r;
        const int nball = cnt[(size_t)e * (L + 2) + L];
        for (int r = 0; r < nball; ++r)
          for (int d = 0; d < dmax; ++d) {
            const int m = idx[(size_t)lst[r] * dmax + d];   // a neighbour of C_L lies in C_{L+1}
            if (pos[m] < 0) return bail(GNA_UNSUPPORTED, "ball table: neighbour outside C_{L+1}");
            tabv.push_back((uint16_t)pos[m]);
          }
        while (tabv.size() % 8) tabv.push_back(0);
        meta[e].y = (int)(tabv.size() - meta[e].x) / 8;
        for (int nd : lst) pos[nd] = -1;
      }
    }
    // bond tables of the pipelined kernels: header |C_0| .. |C_{L+1}|, node ids, then
    // the pool tag (pool << 12 | offset in the pool slot) of every list position and
    // of the neighbour positions of each row of C_L (see gna_pipe.h)
    {
      c->ball_cmax.assign(L + 2, 0);
      c->ball_ringmax.assign(L + 2, 0);
      for (int e = 0; e < E; ++e)
        for (int l = 0; l <= L + 1; ++l) {
          const int* ce = &cnt[(size_t)e * (L + 2)];
          c->ball_cmax[l] = std::max(c->ball_cmax[l], ce[l]);
          if (l >= 3) c->ball_ringmax[l] = std::max(c->ball_ringmax[l], ce[l] - ce[l - 1]);
        }
      const int nbt = max_ball * dmax;
      const int tabw = (kPipeHdr + 2 * r8 + nbt + 7) / 8 * 8;
      bool ok = E > 0 && L >= 1 && L <= kPipeMaxL && N <= 65535 && E <= 65535 && c->ball_cmax[2] < 4096 &&
                tabw <= 8 * 64 * kPipeTabVec;
      for (int sr = 3; sr <= L + 1; ++sr) ok = ok && c->ball_ringmax[sr] < 4096;
      std::vector<uint16_t> pt;
      if (ok) {
        pt.assign((size_t)E * tabw, 0);
        std::vector<int> pos(N, -1);
        for (int e = 0; e < E; ++e) {
          const std::vector<int>& lst = lists[e];
          const int* ce = &cnt[(size_t)e * (L + 2)];
          uint16_t* t = pt.data() + (size_t)e * tabw;
          for (int l = 0; l <= L + 1; ++l) t[l] = (uint16_t)ce[l];
          auto tag = [&](int p) {
            if (p < ce[2]) return (uint16_t)p;   // pool 0: the prefix [0, |C_2|)
            int sr = 3;
            while (p >= ce[sr]) ++sr;            // ring sr: [|C_{sr-1}|, |C_sr|), pool sr - 2
            return (uint16_t)(((sr - 2) << 12) | (p - ce[sr - 1]));
          };
          for (int r = 0; r < r8; ++r) {
            t[kPipeHdr + r] = r < (int)lst.size() ? (uint16_t)lst[r] : (uint16_t)0xffff;
            t[kPipeHdr + r8 + r] = r < (int)lst.size() ? tag(r) : (uint16_t)0;
          }
          for (size_t r = 0; r < lst.size(); ++r) pos[lst[r]] = (int)r;
          for (int r = 0; r < ce[L]; ++r)
            for (int d = 0; d < dmax; ++d)
              t[kPipeHdr + 2 * r8 + r * dmax + d] = tag(pos[idx[(size_t)lst[r] * dmax + d]]);
          for (int nd : lst) pos[nd] = -1;
        }
      }
      c->pipe_ok = ok;
      c->pipe_tabw = tabw;
      if ((st = dev_alloc(c, &c->d_sched, (size_t)2 * kPipeMaxD * kMaxWaves * sizeof(uint2))) ||
          (ok && (st = dev_alloc(c, &c->d_pipe_tab, pt.size() * 2))) ||
          (ok && (st = dev_alloc(c, &c->d_terms, MB * (size_t)std::max(1, E) * 2 * sizeof(double)))))
        return bail(st, c->err);
      if (ok) {
        he = hipMemcpy(c->d_pipe_tab, pt.data(), pt.size() * 2, hipMemcpyHostToDevice);
        if (he != hipSuccess) return bail(GNA_HIP_ERROR, std::string("hipMemcpy: ") + hipGetErrorString(he));
      }
    }
    c->inc_r8 = r8;
    c->inc_max_rows = max_rows;
    c->inc_max_ball = max_ball;
    c->inc_max_tiles = max_tiles;
    c->inc_w_bytes = w_bytes;
    c->lds_max = lds_max;
    {
      // shape signature: N, |E|, degree histogram, F, L, precision
      std::vector<int> hist;
      for (int d : deg) {
        if ((int)hist.size() <= d) hist.resize(d + 1, 0);
        ++hist[d];
      }
      std::string k = std::to_string(N) + "/" + std::to_string(E) + "/";
      for (int h : hist) k += std::to_string(h) + ",";
      k += "/" + std::to_string(F) + "/" + std::to_string(L) + "/" + std::to_string(c->prec);
      c->tune_key = k;
    }
    // default: the largest S that fits, 8 waves; a shape tuned earlier in this
    // process for the same signature wins
    IncTune tt{IncShape{-kIncMaxSwaps, false, 2}, IncShape{-kIncMaxSwaps, false, 2}};
    (void)tune_lookup(c->tune_key, &tt);
    if ((st = inc_configure(c, tt.el, 1)) != GNA_OK || (st = inc_configure(c, tt.sw, 2)) != GNA_OK)
      return bail(st, c->err);
    const size_t plane_bytes = (size_t)g.npad * F * c->sz_Acc;
    if ((st = dev_alloc(c, &c->d_ball_meta, meta.size() * 8)) ||
        (st = dev_alloc(c, &c->d_ball_cnt, cnt.size() * 4)) ||
        (st = dev_alloc(c, &c->d_ball_tab, std::max<size_t>(8, tabv.size()) * 2)) ||
        (st = dev_alloc(c, &c->d_inc_planes, (size_t)MB * 2 * std::max(L, 1) * plane_bytes)))
      return bail(st, c->err);
    he = hipMemcpy(c->d_ball_meta, meta.data(), meta.size() * 8, hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(c->d_ball_cnt, cnt.data(), cnt.size() * 4, hipMemcpyHostToDevice);
    if (he == hipSuccess && !tabv.empty())
      he = hipMemcpy(c->d_ball_tab, tabv.data(), tabv.size() * 2, hipMemcpyHostToDevice);
    if (he != hipSuccess) return bail(GNA_HIP_ERROR, std::string("hipMemcpy: ") + hipGetErrorString(he));
  }
  he = hipMemcpy(c->d_edges, hedges.data(), hedges.size() * 4, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(c->d_idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemcpy(c->d_val64, val.data(), val.size() * 8, hipMemcpyHostToDevice);
  if (he == hipSuccess)
    he = (c->sz_Acc == 8) ? hipMemcpy(c->d_val, val.data(), val.size() * 8, hipMemcpyHostToDevice)
                          : hipMemcpy(c->d_val, val32.data(), val32.size() * 4, hipMemcpyHostToDevice);
  if (he != hipSuccess) return bail(GNA_HIP_ERROR, std::string("hipMemcpy: ") + hipGetErrorString(he));
  *out = c;
  return GNA_OK;
}

void gna_destroy(gna_ctx* ctx) {
  if (!ctx) return;
  // teardown has no status to return: a failure here leaves nothing to undo
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& r : ctx->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  free_all(ctx);
  delete ctx;
}

int64_t gna_num_params(const gna_ctx* ctx) { return ctx ? ctx->P : -1; }

const char* gna_last_error(const gna_ctx* ctx) {
  if (!ctx) {
    std::lock_guard<std::mutex> lk(g_err_mu);
    return g_init_err.c_str();
  }
  return ctx->err.c_str();
}

gna_status gna_set_stream(gna_ctx* ctx, void* stream) {
  if (!ctx) return GNA_INVALID_ARG;
  ctx->stream = reinterpret_cast<hipStream_t>(stream);
  return GNA_OK;
}

static gna_status check_batch(gna_ctx* c, int B) {
  if (B < 0) return fail(c, GNA_INVALID_ARG, "B must be >= 0");
  if (B > c->max_batch) return fail(c, GNA_INVALID_ARG, "B exceeds max_batch");
  return GNA_OK;
}

gna_status gna_logpsi(gna_ctx* c, const double* theta, const int8_t* spins, int32_t B, double* logpsi) {
  if (!c) return GNA_INVALID_ARG;
  if (gna_status st = check_batch(c, B)) return st;
  if (!valid_ptr(theta) || (B > 0 && (!valid_ptr(spins) || !valid_ptr(logpsi))))
    return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  if (B == 0) return GNA_OK;
  if (gna_status st = prepare(c, theta)) return st;
  return run_logpsi(c, theta, spins, B, logpsi);
}

gna_status gna_local_energy(gna_ctx* c, const double* theta, const int8_t* spins, int32_t B, double* eloc,
                            int64_t* n_evals) {
  if (!c) return GNA_INVALID_ARG;
  if (gna_status st = check_batch(c, B)) return st;
  if (!valid_ptr(theta) || (B > 0 && (!valid_ptr(spins) || !valid_ptr(eloc))))
    return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  if (gna_status st = prepare(c, theta)) return st;
  if (c->eloc_mode == GNA_ELOC_FULL)
    if (gna_status st = run_logpsi(c, theta, spins, B, c->d_base)) return st;
  long long* nev = n_evals ? reinterpret_cast<long long*>(n_evals) : c->d_nev;
  return run_eloc(c, theta, spins, B, c->d_base, eloc, nev);
}

gna_status gna_local_energy_noalloc(gna_ctx* c, const double* theta, const int8_t* spins, int32_t B,
                                    double* eloc, int64_t* n_evals) {
  if (!c) return GNA_INVALID_ARG;
  if (gna_status st = check_batch(c, B)) return st;
  if (!valid_ptr(theta) || (B > 0 && (!valid_ptr(spins) || !valid_ptr(eloc))))
    return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  if (!c->scratch_dev) return fail(c, GNA_HIP_ERROR, c->scratch_err);
  // scratch layout (256-byte aligned parts): evaluation counter, base log psi [B][2],
  // per-item partial sums [B * n_chunks][4], per-item counts [B * n_chunks], and with
  // the pipelined local-energy kernel its exchange terms [B][E][2]
  int n_chunks = 1, chunk = 1;
  eloc_chunks(c, std::max(B, 1), &n_chunks, &chunk);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t items = (size_t)B * n_chunks;
  const bool piped = c->eloc_mode == GNA_ELOC_INCREMENTAL && c->pipe_el;
  const size_t off_base = 256;
  const size_t off_part = al(off_base + (size_t)B * 2 * sizeof(double));
  const size_t off_cnt = al(off_part + items * 4 * sizeof(double));
  const size_t off_terms = al(off_cnt + items * sizeof(int));
  const size_t need = piped ? off_terms + (size_t)B * std::max(1, c->E) * 2 * sizeof(double) : off_cnt + items * sizeof(int);
  if (need > kStaticScratchBytes)
    return fail(c, GNA_INVALID_ARG, "gna_local_energy_noalloc: B = " + std::to_string(B) + " needs " +
                                        std::to_string(need) + " bytes of static scratch, above the maximum of " +
                                        std::to_string(kStaticScratchBytes));
  unsigned char* sc = reinterpret_cast<unsigned char*>(c->scratch_dev);
  long long* nev = n_evals ? reinterpret_cast<long long*>(n_evals) : reinterpret_cast<long long*>(sc);
  double* base = reinterpret_cast<double*>(sc + off_base);
  double* partial = reinterpret_cast<double*>(sc + off_part);
  int* cnt = reinterpret_cast<int*>(sc + off_cnt);
  double* terms = piped ? reinterpret_cast<double*>(sc + off_terms) : nullptr;
  if (gna_status st = prepare(c, theta)) return st;
  if (c->eloc_mode == GNA_ELOC_FULL)
    if (gna_status st = run_logpsi(c, theta, spins, B, base)) return st;
  // every item's partial sums and count are written by the kernel that owns the
  // item (every exchange term read is written first); the counter is cleared by a
  // fill kernel inside run_eloc
  return run_eloc(c, theta, spins, B, base, eloc, nev, false, partial, cnt, terms);
}

static gna_status run_sweep(gna_ctx* c, const double* theta, int8_t* spins, double* logpsi, int32_t B,
                            int32_t n_sweeps, uint64_t seed, uint64_t counter_base,
                            const unsigned long long* counter_dev, int32_t* n_accept) {
  if (B == 0) return GNA_OK;
  if (gna_status st = prepare(c, theta)) return st;
  Net net = make_net(c, theta);
  if (c->eloc_mode == GNA_ELOC_INCREMENTAL) {
    // planes of the current configurations, incremental sweeps, then log psi of the
    // final configurations by the full evaluation
    void* planes = c->d_inc_planes;
    double* none = nullptr;
    {
      Timed tm(c, "k_inc_base");
      void* a1[] = {&net, &spins, &B, &planes, &none};
      hipError_t e = hipLaunchKernel(c->ik.base, dim3(std::min(B, c->grid_inc_base)), dim3(64 * c->geo.wpc), a1,
                                     (size_t)c->geo.lds_bytes, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "k_inc_base");
    }
    if (gna_status st = check_launch(c, "k_inc_base")) return st;
    IncNet inc = make_inc(c);
    int Bv = B, ns = n_sweeps;
    unsigned long long sd = seed, cb = counter_base;
    int* acc = n_accept;
    if (c->pipe_sw) {
      PipeGeo pg = c->pgeo_sw;
      const int grid_p = std::max(1, std::min(c->grid_pipe_sw, (B + pg.D - 1) / pg.D));
      const uint2* sched = c->d_sched + (size_t)kPipeMaxD * kMaxWaves;
      const uint16_t* gtab = c->d_pipe_tab;
      {
        Timed tm(c, "k_sweep_pipe");
        void* a2[] = {&net, &inc, &pg, &sched, &gtab, &spins, &planes, &Bv, &ns, &sd, &cb, &counter_dev, &acc};
        hipError_t e = hipLaunchKernel(c->pk_sw.sweep, dim3(grid_p), dim3(64 * pg.nw), a2, (size_t)pg.lds_bytes,
                                       c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "k_sweep_pipe");
      }
      if (gna_status st = check_launch(c, "k_sweep_pipe")) return st;
      return run_logpsi_planes(c, theta, spins, B, logpsi);
    }
    IncGeo ig = c->igeo_sw;
    const int grid_s = std::max(1, std::min(c->grid_sweep_inc, (B + ig.S - 1) / ig.S));
    {
      Timed tm(c, "k_sweep_inc");
      void* a2[] = {&net, &inc, &ig, &spins, &planes, &Bv, &ns, &sd, &cb, &counter_dev, &acc};
      hipError_t e = hipLaunchKernel(c->ik.sweep, dim3(grid_s), dim3(64 * ig.nw), a2, (size_t)ig.lds_bytes, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "k_sweep_inc");
    }
    if (gna_status st = check_launch(c, "k_sweep_inc")) return st;
    return run_logpsi_planes(c, theta, spins, B, logpsi);
  }
  int grid = std::min(B, c->grid_sweep);
  int Bv = B, ns = n_sweeps;
  unsigned long long sd = seed, cb = counter_base;
  int* acc = n_accept;
  void* args[] = {&net, &spins, &logpsi, &Bv, &ns, &sd, &cb, &counter_dev, &acc};
  return launch(c, c->kern.sweep, grid, args, "k_sweep");
}

gna_status gna_metropolis_sweep(gna_ctx* c, const double* theta, int8_t* spins, double* logpsi, int32_t B,
                                int32_t n_sweeps, uint64_t seed, uint64_t counter_base, int32_t* n_accept) {
  if (!c) return GNA_INVALID_ARG;
  if (gna_status st = check_batch(c, B)) return st;
  if (n_sweeps < 0) return fail(c, GNA_INVALID_ARG, "n_sweeps must be >= 0");
  if (!valid_ptr(theta) || (B > 0 && (!valid_ptr(spins) || !valid_ptr(logpsi))))
    return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  if (c->E == 0 && n_sweeps > 0) return fail(c, GNA_INVALID_ARG, "graph has no bonds to propose");
  return run_sweep(c, theta, spins, logpsi, B, n_sweeps, seed, counter_base, nullptr, n_accept);
}

gna_status gna_logpsi_vjp(gna_ctx* c, const double* theta, const int8_t* spins, int32_t B, const double* cot,
                          double* grad) {
  if (!c) return GNA_INVALID_ARG;
  if (gna_status st = check_batch(c, B)) return st;
  if (!valid_ptr(theta) || !valid_ptr(grad) || (B > 0 && (!valid_ptr(spins) || !valid_ptr(cot))))
    return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  return run_vjp(c, theta, spins, B, cot, grad);
}

// One ISGO update's gradient.  base_ready (incremental mode only): log psi of the
// configurations under theta, with the planes holding their base pass (as an
// incremental sweep under the same theta leaves them); the base pass is skipped.
static gna_status isgo_impl(gna_ctx* c, const double* theta, const int8_t* spins, const double* logpsi_old,
                            const double* counts, int32_t B, double* grad, double* stats, double* eloc,
                            const double* base_ready) {
  if (gna_status st = prepare(c, theta)) return st;
  if (c->eloc_mode == GNA_ELOC_FULL)   // the incremental base pass writes log psi itself
    if (gna_status st = run_logpsi(c, theta, spins, B, c->d_base)) return st;
  const double* base = base_ready ? base_ready : c->d_base;
  double* el = eloc ? eloc : c->d_eloc;
  if (gna_status st = run_eloc(c, theta, spins, B, base, el, c->d_nev, base_ready != nullptr)) return st;
  {
    Timed tm(c, "k_isgo_stats");
    hipLaunchKernelGGL(k_isgo_stats, dim3(1), dim3(kStatThreads), 0, c->stream, B, logpsi_old, base, el,
                     counts, c->d_nev, stats, c->d_cot);
  }
  if (gna_status st = check_launch(c, "k_isgo_stats")) return st;
  return run_vjp(c, theta, spins, B, c->d_cot, grad);
}

gna_status gna_isgo_grad(gna_ctx* c, const double* theta, const int8_t* spins, const double* logpsi_old,
                         const double* counts, int32_t B, double* grad, double* stats, double* eloc) {
  if (!c) return GNA_INVALID_ARG;
  if (gna_status st = check_batch(c, B)) return st;
  if (!valid_ptr(theta) || !valid_ptr(grad) || !valid_ptr(stats) ||
      (B > 0 && (!valid_ptr(spins) || !valid_ptr(logpsi_old))))
    return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  return isgo_impl(c, theta, spins, logpsi_old, counts, B, grad, stats, eloc, nullptr);
}

gna_status gna_sgd_update(gna_ctx* c, double* theta, const double* grad, double alpha) {
  if (!c) return GNA_INVALID_ARG;
  if (!valid_ptr(theta) || !valid_ptr(grad)) return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  if (!std::isfinite(alpha)) return fail(c, GNA_INVALID_ARG, "alpha must be finite");
  const int n = (int)c->P;
  Timed tm(c, "k_sgd");
  hipLaunchKernelGGL(k_sgd, dim3((n + 255) / 256), dim3(256), 0, c->stream, theta, grad, alpha, n);
  return check_launch(c, "k_sgd");
}

gna_status gna_step(gna_ctx* c, double* theta, int8_t* spins, double* logpsi, int32_t B, int32_t n_sweeps,
                    uint64_t seed, uint64_t* counter, double lr, double* grad, double* stats, double* eloc,
                    int32_t* n_accept) {
  if (!c) return GNA_INVALID_ARG;
  if (gna_status st = check_batch(c, B)) return st;
  if (n_sweeps < 0) return fail(c, GNA_INVALID_ARG, "n_sweeps must be >= 0");
  if (!std::isfinite(lr)) return fail(c, GNA_INVALID_ARG, "lr must be finite");
  if (!valid_ptr(theta) || !valid_ptr(counter) || !valid_ptr(grad) || !valid_ptr(stats) ||
      (B > 0 && (!valid_ptr(spins) || !valid_ptr(logpsi))))
    return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  if (c->E == 0 && n_sweeps > 0) return fail(c, GNA_INVALID_ARG, "graph has no bonds to propose");
  if (gna_status st = prepare(c, theta)) return st;
  const bool inc = c->eloc_mode == GNA_ELOC_INCREMENTAL;
  // the full sampler starts from log psi of the chains; the incremental one evaluates
  // the final configurations itself and leaves their base pass in the planes
  if (!inc)
    if (gna_status st = run_logpsi(c, theta, spins, B, logpsi)) return st;
  unsigned long long* cd = reinterpret_cast<unsigned long long*>(counter);
  if (gna_status st = run_sweep(c, theta, spins, logpsi, B, n_sweeps, seed, 0, cd, n_accept)) return st;
  {
    Timed tm(c, "k_add_u64");
    hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(64), 0, c->stream, cd,
                       (unsigned long long)n_sweeps * (unsigned long long)c->N);
  }
  if (gna_status st = check_launch(c, "k_add_u64")) return st;
  // theta is unchanged since the sweep: its samples' log psi is the new log psi, and
  // in incremental mode the planes are already the base pass of the local energy
  if (gna_status st = isgo_impl(c, theta, spins, logpsi, nullptr, B, grad, stats, eloc, inc ? logpsi : nullptr))
    return st;
  return gna_sgd_update(c, theta, grad, lr);
}

gna_status gna_autotune(gna_ctx* c, const double* theta, const int8_t* spins, int32_t B, int32_t* chosen) {
  if (!c) return GNA_INVALID_ARG;
  if (gna_status st = check_batch(c, B)) return st;
  if (B < 1) return fail(c, GNA_INVALID_ARG, "autotune needs B >= 1");
  if (!valid_ptr(theta) || !valid_ptr(spins)) return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  if (c->eloc_mode != GNA_ELOC_INCREMENTAL) {   // the full evaluator's shape is fixed at init
    if (chosen)
      for (int k = 0; k < 8; ++k) chosen[k] = 0;
    return GNA_OK;
  }
  if (gna_status st = prepare(c, theta)) return st;
  const IncShape before = shape_el(c);
  const IncShape before_sw = shape_sw(c);
  // candidates: the four largest S that fit, both wave shapes, one or two samples per XCD
  std::vector<IncShape> cand;
  int smax = 0;
  for (int S = kIncMaxSwaps; S >= 1 && !smax; --S)
    if (inc_configure(c, IncShape{S, false, 2}, 1) == GNA_OK) smax = S;
  for (int px = 1; px <= 2; ++px) {   // the layer-pipelined kernels, 8 or 16 waves
    cand.push_back(IncShape{0, false, px, 0});
    cand.push_back(IncShape{0, true, px, 0});
  }
  for (int S = smax; S >= 1 && S > smax - 4; --S)
    for (int px = 1; px <= 2; ++px) {
      cand.push_back(IncShape{S, true, px, 0});
      // 8 waves, and fewer waves where that evens out the tiles per wave
      const int tiles = S * c->inc_max_tiles;
      for (int nw = kMaxWaves / 2; nw >= 5; --nw)
        if (nw == kMaxWaves / 2 || (tiles + nw - 1) / nw == (tiles + kMaxWaves / 2 - 1) / (kMaxWaves / 2))
          cand.push_back(IncShape{S, false, px, nw});
    }
  // the sweep runs on a copy of the batch (it moves the chains); these buffers live
  // for the call only
  int8_t* tsp = nullptr;
  double* tlp = nullptr;
  int32_t* tacc = nullptr;
  if (hipMalloc(&tsp, (size_t)B * c->N) != hipSuccess || hipMalloc(&tlp, (size_t)B * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc(&tacc, (size_t)B * sizeof(int32_t)) != hipSuccess) {
    (void)hipFree(tsp);
    (void)hipFree(tlp);
    (void)hipFree(tacc);
    (void)inc_configure(c, before, 1);
    return fail(c, GNA_OUT_OF_MEMORY, "autotune: temporary batch copy");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipFree(tsp);
    (void)hipFree(tlp);
    (void)hipFree(tacc);
    (void)inc_configure(c, before, 1);
    return fail(c, GNA_HIP_ERROR, "hipEventCreate failed");
  }
  const bool prof = c->prof_on;
  c->prof_on = false;
  gna_status st = GNA_OK;
  // time `run` (warm-up, then two timed calls) under every candidate of `which`
  auto tune = [&](int which, auto&& run, IncShape* best, float* best_ms) {
    *best_ms = -1.f;
    for (const IncShape& sh : cand) {
      if (which == 2 && sh.per_xcd != 1) continue;   // the sweep has no per-XCD sample split
      if (inc_configure(c, sh, which) != GNA_OK) continue;
      if ((st = run()) != GNA_OK) return;   // warm
      if (hipEventRecord(e0, c->stream) != hipSuccess) {
        st = fail(c, GNA_HIP_ERROR, "hipEventRecord failed");
        return;
      }
      for (int r = 0; r < 2 && st == GNA_OK; ++r) st = run();
      if (st != GNA_OK) return;
      if (hipEventRecord(e1, c->stream) != hipSuccess) {
        st = fail(c, GNA_HIP_ERROR, "hipEventRecord failed");
        return;
      }
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = fail(c, GNA_HIP_ERROR, "hipEventSynchronize failed");
        return;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(c, GNA_HIP_ERROR, "hipEventElapsedTime failed");
        return;
      }
      if (*best_ms < 0.f || ms < *best_ms) {
        *best_ms = ms;
        *best = sh;
      }
    }
  };
  IncShape best = before, best_sw = before_sw;
  float ms_el = -1.f, ms_sw = -1.f;
  tune(1, [&] { return run_eloc(c, theta, spins, B, c->d_base, c->d_eloc, c->d_nev); }, &best, &ms_el);
  if (st == GNA_OK && (st = inc_configure(c, best, 1)) == GNA_OK)
    tune(2, [&] {
      if (hipMemcpyAsync(tsp, spins, (size_t)B * c->N, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return fail(c, GNA_HIP_ERROR, "autotune: batch copy");
      return run_sweep(c, theta, tsp, tlp, B, 1, 0, 0, nullptr, tacc);
    }, &best_sw, &ms_sw);
  if (st == GNA_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = fail(c, GNA_HIP_ERROR, "autotune sync");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(tsp);
  (void)hipFree(tlp);
  (void)hipFree(tacc);
  c->prof_on = prof;
  if (st != GNA_OK) {
    (void)inc_configure(c, before, 1);
    (void)inc_configure(c, before_sw, 2);
    return st;
  }
  if ((st = inc_configure(c, best, 1)) != GNA_OK || (st = inc_configure(c, best_sw, 2)) != GNA_OK) return st;
  tune_store(c->tune_key, IncTune{best, best_sw});
  if (chosen) {
    chosen[0] = best.S;   // 0: the pipelined kernel
    chosen[1] = c->pipe_el ? c->pgeo_el.nw : (c->inc_wide ? kMaxWaves : c->igeo.nw);   // 16: the 1024-thread variant
    chosen[2] = best.per_xcd;
    chosen[3] = (int32_t)(ms_el * 500.f);   // microseconds per local-energy call
    chosen[4] = best_sw.S;
    chosen[5] = c->pipe_sw ? c->pgeo_sw.nw : (c->inc_sw_wide ? kMaxWaves : c->igeo_sw.nw);
    chosen[6] = c->inc_sw_maxt;
    chosen[7] = (int32_t)(ms_sw * 500.f);   // microseconds per one-sweep call
  }
  return GNA_OK;
}

gna_status gna_set_shape(gna_ctx* c, int32_t which, int32_t jobs_in_flight, int32_t waves, int32_t samples_per_xcd) {
  if (!c) return GNA_INVALID_ARG;
  if (c->eloc_mode != GNA_ELOC_INCREMENTAL)
    return fail(c, GNA_INVALID_ARG, "kernel shapes apply to the incremental mode only");
  if (which < 1 || which > 3) return fail(c, GNA_INVALID_ARG, "which must be 1 (local energy), 2 (sweep) or 3");
  if (jobs_in_flight < 0 || jobs_in_flight > kIncMaxSwaps)
    return fail(c, GNA_INVALID_ARG, "jobs_in_flight must be 0 (pipelined) or in [1, 8]");
  if (waves != kMaxWaves && (waves < 1 || waves > kMaxWaves / 2))
    return fail(c, GNA_INVALID_ARG, "waves must be 16 or in [1, 8]");
  if (jobs_in_flight == 0 && waves != kMaxWaves && waves != kMaxWaves / 2)
    return fail(c, GNA_INVALID_ARG, "the pipelined kernels take 8 or 16 waves");
  if (samples_per_xcd < 1 || samples_per_xcd > 8) return fail(c, GNA_INVALID_ARG, "samples_per_xcd must be in [1, 8]");
  const IncShape before = shape_el(c);
  const IncShape before_sw = shape_sw(c);
  const bool wide = waves == kMaxWaves;
  const IncShape sh{jobs_in_flight, wide, samples_per_xcd, (wide || jobs_in_flight == 0) ? 0 : waves};
  gna_status st = GNA_OK;
  if (which & 1) st = inc_configure(c, sh, 1);
  if (st == GNA_OK && (which & 2)) st = inc_configure(c, sh, 2);
  if (st != GNA_OK) {
    std::string msg = c->err;
    (void)inc_configure(c, before, 1);
    (void)inc_configure(c, before_sw, 2);
    return fail(c, st, msg.c_str());
  }
  return GNA_OK;
}

gna_status gna_group_duplicates(gna_ctx* c, const int8_t* spins, int32_t B, int8_t* uniq, double* counts,
                                int32_t* n_unique) {
  if (!c) return GNA_INVALID_ARG;
  if (gna_status st = check_batch(c, B)) return st;
  if (!valid_ptr(n_unique) || (B > 0 && (!valid_ptr(spins) || !valid_ptr(uniq) || !valid_ptr(counts))))
    return fail(c, GNA_INVALID_ARG, "NULL pointer argument");
  if (B > 0 && (const void*)uniq == (const void*)spins) return fail(c, GNA_INVALID_ARG, "uniq must not alias spins");
  const int n = c->N, T = c->grp_T;
  int* slot = c->d_grp_row;
  int* rep = slot + c->max_batch;
  int* gid = rep + c->max_batch;
  int* cnt = gid + c->max_batch;
  const int wpb = 4;                              // rows (waves) per 256-thread workgroup
  const int rb = std::max(1, (B + wpb - 1) / wpb);
  {
    Timed tm(c, "k_group");
    hipLaunchKernelGGL(k_group_clear, dim3(std::min(1024, (T + 255) / 256)), dim3(256), 0, c->stream, c->d_grp_key,
                       c->d_grp_val, T, cnt, (int)B);
    if (B > 0) {
      hipLaunchKernelGGL(k_group_insert, dim3(rb), dim3(64 * wpb), 0, c->stream, spins, n, (int)B, c->d_grp_key,
                         c->d_grp_val, T, slot);
      hipLaunchKernelGGL(k_group_rep, dim3(rb), dim3(64 * wpb), 0, c->stream, spins, n, (int)B, c->d_grp_val, slot,
                         rep);
    }
    hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(1024), 0, c->stream, rep, (int)B, gid, n_unique);
    if (B > 0) {
      hipLaunchKernelGGL(k_group_scatter, dim3(rb), dim3(64 * wpb), 0, c->stream, spins, n, (int)B, rep, gid, cnt,
                         uniq);
      hipLaunchKernelGGL(k_group_finish, dim3(rb), dim3(64 * wpb), 0, c->stream, cnt, n_unique, n, (int)B, counts,
                         uniq);
    }
  }
  return check_launch(c, "k_group");
}

int32_t gna_config_info(const gna_ctx* c, int32_t* info, int32_t n) {
  if (!c || (n > 0 && !info)) return -1;
  const bool inc = c->eloc_mode == GNA_ELOC_INCREMENTAL;
  // waves: 16 names the one-tile-per-wave variant (it launches one wave per tile, at most 16)
  const int el_s = c->pipe_el ? 0 : c->igeo.S, sw_s = c->pipe_sw ? 0 : c->igeo_sw.S;
  const int el_w = c->pipe_el ? c->pgeo_el.nw : (c->inc_wide ? kMaxWaves : c->igeo.nw);
  const int sw_w = c->pipe_sw ? c->pgeo_sw.nw : (c->inc_sw_wide ? kMaxWaves : c->igeo_sw.nw);
  const int32_t v[11] = {c->eloc_mode, inc ? el_s : 0, inc ? el_w : c->geo.wpc,
                         inc ? c->inc_maxt : c->tpw, inc ? c->inc_per_xcd : 0, c->prec, c->F, c->L,
                         inc ? sw_s : 0, inc ? sw_w : c->geo.wpc,
                         inc ? c->inc_sw_maxt : c->tpw};
  for (int k = 0; k < n && k < 11; ++k) info[k] = v[k];
  return 11;
}

gna_status gna_set_couplings(gna_ctx* c, double jz, double jxy, double hb, double cb) {
  if (!c) return GNA_INVALID_ARG;
  if (!std::isfinite(jz) || !std::isfinite(jxy) || !std::isfinite(hb) || !std::isfinite(cb))
    return fail(c, GNA_INVALID_ARG, "couplings must be finite");
  c->jz = jz;
  c->jxy = jxy;
  c->hb = hb;
  c->cb = cb;
  return GNA_OK;
}

gna_status gna_profile_enable(gna_ctx* c, int32_t on) {
  if (!c) return GNA_INVALID_ARG;
  c->prof_on = (on != 0);
  return GNA_OK;
}

int32_t gna_profile_read(gna_ctx* c, int32_t max_entries, char* names, int64_t* launches, double* total_ms) {
  if (!c || max_entries < 0 || (max_entries > 0 && (!names || !launches || !total_ms))) return -1;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return -1;
  bool bad = c->prof_err;
  c->prof_err = false;
  std::vector<std::pair<std::string, std::pair<int64_t, double>>> agg;
  for (auto& r : c->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) bad = true;
    size_t k = 0;
    while (k < agg.size() && agg[k].first != r.name) ++k;
    if (k == agg.size()) agg.push_back({r.name, {0, 0.0}});
    agg[k].second.first += 1;
    agg[k].second.second += ms;
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->recs.clear();
  if (bad) {
    c->err = "kernel timing: an event could not be created, recorded or read";
    return -1;
  }
  const int n = (int)agg.size();
  for (int k = 0; k < n && k < max_entries; ++k) {
    std::strncpy(names + 64 * k, agg[k].first.c_str(), 63);
    names[64 * k + 63] = 0;
    launches[k] = agg[k].second.first;
    total_ms[k] = agg[k].second.second;
  }
  return n;
}

}  // extern "C"
