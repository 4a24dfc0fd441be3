// Reverse pass of the ansatz (gna_logpsi_vjp, gna_isgo_grad) on MFMA.
//
// For a chunk of samples the forward pass is recomputed once and its per-layer
// inputs H^l and messages M^l are kept as planes (npad x F, slot order, see
// eval_config).  Then, layer by layer from the top, with P = [M | H] W + b and
// H' = f(P):
//   dP   = dH' * (1 - H'^2)         (tanh; ReLU + layer normalisation: its VJP)
//   dW  += [M | H]^T dP           (k_vjp_dw: rows of all samples are the
//   db  += sum_rows dP             MFMA reduction dimension)
//   dX   = dP W^T                  (k_vjp_dx: per sample, same register layout
//   dH   = dX_self + A_hat dX_msg   as the forward; A_hat is symmetric)
// and finally the embedding and head gradients (k_vjp_tail).  Every workgroup
// accumulates into its own FP64 row of `part`; k_vjp_reduce adds the rows in
// order, so the result does not depend on timing.
#pragma once

#include <type_traits>

#include "gna_kernels.h"

namespace gna {

struct VNet {
  int n, F, L, tied, dmax, npad, ntiles, wpc;
  int act;               // 0: tanh, 1: ReLU + layer normalisation
  const int* ell_idx;    // [npad][dmax]
  const void* ell_val;   // [npad][dmax], Acc
  const void* wbwd;      // [nW][2F/16][F/4][64] fragments of W (not transposed), Acc
  const double* theta;   // FP64 parameters (heads are read from here)
  int npar;
  size_t plane;          // npad * F
  int nplanes;           // planes per sample: 2L+1 forward + dP + dXm + dH(2) [+ Y^1..Y^L]
};

// planes of one sample: 0..L = H^l, L+1..2L = M^l, then dP, dXm, dH0, dH1 and,
// with ReLU + layer normalisation, Y^1..Y^L
__device__ __forceinline__ int plane_dP(const VNet& v) { return 2 * v.L + 1; }
__device__ __forceinline__ int plane_dXm(const VNet& v) { return 2 * v.L + 2; }
__device__ __forceinline__ int plane_dH(const VNet& v, int which) { return 2 * v.L + 3 + (which & 1); }
// post-ReLU rows Y^l (l = 1..L) of ReLU + layer normalisation
__device__ __forceinline__ int plane_Y(const VNet& v, int l) { return 2 * v.L + 4 + l; }

// Build the backward fragments: A[m = input feature][kd = output feature] = W,
// fragment (w, tm, s, lane) = W[part*F + row_feature(16 (tm mod F/16) + lane%16)][4s + lane/16]
// with part = tm / (F/16) (0: message rows, 1: self rows).  KS = 4, VEC = 1.
template <class P, int F>
__global__ void k_prepare_bwd(const double* __restrict__ theta, int nW, typename P::Acc* __restrict__ out) {
  constexpr int MT = F / 16, KSB = F / 4;
  const double* W = theta + 3 * F;
  const int per = 2 * MT * KSB * 64;   // = 2 F F
  const int total = nW * per;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    int r = e;
    const int lane = r % 64; r /= 64;
    const int s = r % KSB; r /= KSB;
    const int tm = r % (2 * MT); r /= (2 * MT);
    const int w = r;
    const int part = tm / MT;
    const int k = part * F + P::row_feature(16 * (tm % MT) + lane % 16);
    const int f = 4 * s + lane / 16;
    out[e] = (typename P::Acc)W[(size_t)w * 2 * F * F + (size_t)k * F + f];
  }
}

// Forward recompute storing the planes of samples [b0, b0 + Bc).
template <class P, int F, int TPW, int NCH>
__global__ __launch_bounds__(512) void k_vjp_fwd(Net net, const int8_t* __restrict__ spins,
                                                                   int b0, int Bc, typename P::Acc* planes,
                                                                   int nplanes) {
  extern __shared__ __align__(16) unsigned char smem[];
  Smem<P> s(net.g, smem);
  stage_graph<P>(net, s);
  if (net.tied) stage_weights<P, F>(net, s, 0);
  __syncthreads();
  const size_t per = (size_t)nplanes * net.g.npad * F;
  for (int b = blockIdx.x; b < Bc; b += gridDim.x) {
    load_spins<P>(net, s, spins + (size_t)(b0 + b) * net.n);
    double la = 0, ph = 0;
    eval_config<P, F, TPW, NCH, 1>(net, s, -1, -1, la, ph, planes + b * per);
  }
}

// One layer of the reverse pass for samples [b0, b0 + Bc): dP, dX = dP W^T, and
// dH of the layer input.  layer == L-1 seeds dH^L from the cotangents.
template <class P, int F, int TPW>
__global__ __launch_bounds__(512) void k_vjp_dx(VNet v, int layer, int b0, int Bc,
                                                                  const double* __restrict__ cot,
                                                                  typename P::Acc* planes) {
  using Acc = typename P::Acc;
  using CF = typename P::CF;
  constexpr int NS = F / 4, MT = F / 16, KSB = F / 4;
  extern __shared__ __align__(16) unsigned char smem[];
  Acc* wfr = reinterpret_cast<Acc*>(smem);   // one layer of backward fragments
  // the adjacency (ELL: A_hat value and neighbour of each node and slot), the same
  // for every sample
  Acc* sval = wfr + 2 * F * F;
  int* sidx = reinterpret_cast<int*>(sval + (size_t)v.npad * v.dmax);
  const int wi = v.tied ? 0 : layer;
  {
    const Acc* src = reinterpret_cast<const Acc*>(v.wbwd) + (size_t)wi * 2 * F * F;
    for (int k = threadIdx.x; k < 2 * F * F; k += blockDim.x) wfr[k] = src[k];
    const Acc* ev = reinterpret_cast<const Acc*>(v.ell_val);
    for (int k = threadIdx.x; k < v.npad * v.dmax; k += blockDim.x) {
      sval[k] = ev[k];
      sidx[k] = v.ell_idx[k];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, q = lane >> 4, col = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar branches
  const size_t per = (size_t)v.nplanes * v.plane;
  const int nW = v.tied ? 1 : v.L;
  const double* head_a = v.theta + 3 * F + (size_t)nW * (2 * F * F + F);
  const double* head_p = head_a + F + 3;
  // neighbour rows requested together in the dX_msg sum (fewer with FP64 rows)
  constexpr int NB = sizeof(Acc) == 8 ? 1 : 4;
  for (int b = blockIdx.x; b < Bc; b += gridDim.x) {
    Acc* pb = planes + b * per;
    const Acc* Hout = pb + (size_t)(layer + 1) * v.plane;
    const Acc* dHin = pb + (size_t)plane_dH(v, layer + 1) * v.plane;
    Acc* dHout = pb + (size_t)plane_dH(v, layer) * v.plane;
    Acc* dPp = pb + (size_t)plane_dP(v) * v.plane;
    Acc* dXm = pb + (size_t)plane_dXm(v) * v.plane;
    const double ca = cot[2 * (size_t)(b0 + b)], cp = cot[2 * (size_t)(b0 + b) + 1];
    Acc dxs[TPW][NS];
    // with FP32 rows the next tile's H' and dH' are requested before this tile's
    // products (FP64 rows have no registers for it)
    constexpr bool kPre = sizeof(Acc) == 4;
    const bool top = layer == v.L - 1;
    Acc hn_n[NS], dh_n[NS];
    auto fetch = [&](int k) {
      const int tile = wv + k * v.wpc;
      if (tile >= v.ntiles) return;
      const size_t off = (size_t)(tile * 16 + col) * F + q * NS;
      lds_read<Acc, NS>(Hout + off, hn_n);
      if (!top) {
        lds_read<Acc, NS>(dHin + off, dh_n);
      } else {
#pragma unroll
        for (int i = 0; i < NS; ++i) dh_n[i] = (Acc)0;   // seeded from the cotangents below
      }
    };
    if (kPre) fetch(0);
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
      const int tile = wv + k * v.wpc;
      if (tile >= v.ntiles) continue;
      const int node = tile * 16 + col;
      const bool real = node < v.n;
      const size_t off = (size_t)node * F + q * NS;
      Acc hn[NS], dh[NS], dp[NS];
      if (!kPre) fetch(k);
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        hn[i] = hn_n[i];
        dh[i] = dh_n[i];
      }
      if (kPre && k + 1 < TPW) fetch(k + 1);
      if (top) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const int f = P::lc(q, i);
          dh[i] = (Acc)(ca * head_a[f] + cp * head_p[f]);
        }
      }
      if (v.act == 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) dp[i] = real ? dh[i] * ((Acc)1 - hn[i] * hn[i]) : (Acc)0;
      } else {   // tile is wave-uniform: the four lanes of a row are active together
        Acc y[NS];
        lds_read<Acc, NS>(pb + (size_t)plane_Y(v, layer + 1) * v.plane + off, y);
        relu_ln_vjp<Acc, NS>(y, hn, dh, dp);
#pragma unroll
        for (int i = 0; i < NS; ++i) dp[i] = real ? dp[i] : (Acc)0;
      }
      lds_write<Acc, NS>(dPp + off, dp);
      CF dx[2 * MT];
#pragma unroll
      for (int t = 0; t < 2 * MT; ++t) dx[t] = CF{0, 0, 0, 0};
#pragma unroll
      for (int st = 0; st < KSB; ++st) {
#pragma unroll
        for (int t = 0; t < 2 * MT; ++t) {
          dx[t] = P::mma(wfr[(t * KSB + st) * 64 + lane], dp[st], dx[t]);
        }
      }
      Acc xm[NS];
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          xm[4 * t + r] = dx[t][r];
          dxs[k][4 * t + r] = dx[MT + t][r];
        }
      lds_write<Acc, NS>(dXm + off, xm);
    }
    __syncthreads();   // dX_msg of every node of the sample is written
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
      const int tile = wv + k * v.wpc;
      if (tile >= v.ntiles) continue;
      const int node = tile * 16 + col;
      Acc acc[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) acc[i] = dxs[k][i];
      if (node < v.n) {
        const int* ip = sidx + node * v.dmax;
        const Acc* vp = sval + node * v.dmax;
        // the sum in neighbour order; NB rows in flight at a time
        int d = 0;
        for (; d + NB <= v.dmax; d += NB) {
          Acc row[NB][NS];
#pragma unroll
          for (int u = 0; u < NB; ++u) lds_read<Acc, NS>(dXm + (size_t)ip[d + u] * F + q * NS, row[u]);
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            const Acc a = vp[d + u];
#pragma unroll
            for (int i = 0; i < NS; ++i) acc[i] += a * row[u][i];
          }
        }
        for (; d < v.dmax; ++d) {
          const Acc a = vp[d];
          Acc row[NS];
          lds_read<Acc, NS>(dXm + (size_t)ip[d] * F + q * NS, row);
#pragma unroll
          for (int i = 0; i < NS; ++i) acc[i] += a * row[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < NS; ++i) acc[i] = (Acc)0;
      }
      lds_write<Acc, NS>(dHout + (size_t)node * F + q * NS, acc);
    }
    __syncthreads();   // before the next sample reuses nothing, but keep waves in step
  }
}

// dW += [M | H]^T dP and db += sum dP over every row of the chunk (npad rows
// per sample).  256 threads; wave w owns output m-tiles {w, w+4, ...} of the
// 2F x F product and all F/16 n-tiles.  Results go to this workgroup's row of
// `part` (FP64, theta layout) at the logical feature positions.
template <class P, int F>
__global__ __launch_bounds__(256) void k_vjp_dw(VNet v, int layer, int Bc, const typename P::Acc* planes,
                                                double* __restrict__ part) {
  using Acc = typename P::Acc;
  using CF = typename P::CF;
  constexpr int NS = F / 4, MT = F / 16, MTW = (2 * MT + 3) / 4;
  const int lane = threadIdx.x & 63, q = lane >> 4, col = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform: scalar branches
  const size_t per = (size_t)v.nplanes * v.plane;
  const int rows_per_sample = v.npad;
  const long long total_steps = (long long)Bc * rows_per_sample / 4;   // npad is a multiple of 16
  const long long s0 = total_steps * blockIdx.x / gridDim.x;
  const long long s1 = total_steps * (blockIdx.x + 1) / gridDim.x;
  CF acc[MTW][MT];
#pragma unroll
  for (int a = 0; a < MTW; ++a)
#pragma unroll
    for (int t = 0; t < MT; ++t) acc[a][t] = CF{0, 0, 0, 0};
  Acc dbp[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) dbp[t] = (Acc)0;
  // sample and first row of the current 4-row k-step, advanced without division
  // (npad is a multiple of 16, so a k-step never straddles two samples)
  int sb = (int)((s0 * 4) / rows_per_sample), node0 = (int)((s0 * 4) % rows_per_sample);
  // m-tiles of this wave; with 2F/16 a multiple of 4 every wave has MTW of them
  constexpr bool ALL_M = (2 * MT) % 4 == 0;
  // U k-steps per round: all their loads are issued before their MFMAs
  constexpr int U = sizeof(Acc) == 4 ? 8 : 4;
  auto round = [&](auto u_const) {
    constexpr int UU = decltype(u_const)::value;
    Acc bf[UU][MT], af[UU][MTW];
#pragma unroll
    for (int u = 0; u < UU; ++u) {
      const Acc* pb = planes + (size_t)sb * per;
      const size_t off = (size_t)(node0 + q) * F;     // this lane's row of the k-step
      node0 += 4;
      const bool wrap = node0 == rows_per_sample;
      sb += wrap ? 1 : 0;
      node0 = wrap ? 0 : node0;
#pragma unroll
      for (int t = 0; t < MT; ++t) bf[u][t] = pb[(size_t)plane_dP(v) * v.plane + off + 16 * t + col];
#pragma unroll
      for (int a = 0; a < MTW; ++a) {
        const int tm = wv + 4 * a;
        const int pl = (tm < MT) ? (v.L + 1 + layer) : layer;   // M^l or H^l
        af[u][a] = (ALL_M || tm < 2 * MT) ? pb[(size_t)pl * v.plane + off + 16 * (tm % MT) + col] : (Acc)0;
      }
    }
#pragma unroll
    for (int u = 0; u < UU; ++u) {
#pragma unroll
      for (int t = 0; t < MT; ++t) dbp[t] += bf[u][t];
#pragma unroll
      for (int a = 0; a < MTW; ++a) {
        if (!ALL_M && wv + 4 * a >= 2 * MT) continue;   // wave-uniform
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[a][t] = P::mma(af[u][a], bf[u][t], acc[a][t]);
      }
    }
  };
  long long st = s0;
  for (; st + U <= s1; st += U) round(std::integral_constant<int, U>{});
  for (; st < s1; ++st) round(std::integral_constant<int, 1>{});
  // scatter to theta layout: position p = qq*NS + i holds logical feature lc(qq, i)
  double* g = part + (size_t)blockIdx.x * v.npar;
  const int wi = v.tied ? 0 : layer;
  const int nW = v.tied ? 1 : v.L;
  double* gW = g + 3 * F + (size_t)wi * 2 * F * F;
  double* gb = g + 3 * F + (size_t)nW * 2 * F * F + (size_t)wi * F;
  auto logical = [](int p) { return P::lc(p / NS, p % NS); };
#pragma unroll
  for (int a = 0; a < MTW; ++a) {
    const int tm = wv + 4 * a;
    if (tm >= 2 * MT) break;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // D layout: f32 row 4q + r, f64 row 4r + q; column col
        const int mrow = (sizeof(Acc) == 8) ? (4 * r + q) : (4 * q + r);
        const int px = 16 * (tm % MT) + mrow, pd = 16 * t + col;
        const int kx = (tm / MT) * F + logical(px), fd = logical(pd);
        gW[(size_t)kx * F + fd] += (double)acc[a][t][r];
      }
  }
  if (wv == 0) {
    // reduce the four lane groups (rows) of db
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      double x = (double)dbp[t];
      x += __shfl_xor(x, 16, 64);
      x += __shfl_xor(x, 32, 64);
      if (q == 0) gb[logical(16 * t + col)] += x;
    }
  }
}

// Embedding and head gradients for samples [b0, b0 + Bc): per workgroup
// (F threads per feature position, rows strided over the block).
template <class P, int F>
__global__ __launch_bounds__(256) void k_vjp_tail(VNet v, int b0, int Bc, const int8_t* __restrict__ spins,
                                                  const double* __restrict__ cot,
                                                  const typename P::Acc* planes, double* __restrict__ part) {
  using Acc = typename P::Acc;
  constexpr int NS = F / 4;
  const size_t per = (size_t)v.nplanes * v.plane;
  const int p = threadIdx.x % F;           // feature position
  const int rs = threadIdx.x / F, nrs = blockDim.x / F;
  double e0 = 0, e1 = 0, za = 0, zp = 0;
  double ua = 0, up = 0, sca = 0, scp = 0;   // one-hot part: sum c * #up over this thread's nodes
  for (int b = blockIdx.x; b < Bc; b += gridDim.x) {
    const Acc* pb = planes + b * per;
    const Acc* H0 = pb;
    const Acc* HL = pb + (size_t)v.L * v.plane;
    const Acc* dH0 = pb + (size_t)plane_dH(v, 0) * v.plane;
    const int8_t* sb = spins + (size_t)(b0 + b) * v.n;
    const double ca = cot[2 * (size_t)(b0 + b)], cp = cot[2 * (size_t)(b0 + b) + 1];
    // without layers the readout sees H^0 directly: dH^0 = ca v_a + cp v_p
    const int nW0 = v.tied ? 1 : v.L;
    const double* ha = v.theta + 3 * F + (size_t)nW0 * (2 * F * F + F);
    const int fl = P::lc(p / NS, p % NS);
    const double dz = ca * ha[fl] + cp * ha[F + 3 + fl];
    double z = 0;
    int nup = 0;
    auto one = [&](int8_t s, Acc dh, Acc h, Acc hl) {
      nup += s > 0;
      const double dh0 = v.L > 0 ? (double)dh : dz;
      double dp0;
      if (v.act == 0) {
        const double h0 = (double)h;
        dp0 = dh0 * (1.0 - h0 * h0);
      } else {   // the embedding row depends on the spin only: its VJP is applied to the sums
        dp0 = dh0;
      }
      if (s > 0) e1 += dp0; else e0 += dp0;
      z += (double)hl;
    };
    // this thread's nodes in order, eight requested at a time
    constexpr int NU = 8;
    int node = rs;
    for (; node + (NU - 1) * nrs < v.n; node += NU * nrs) {
      int8_t sv[NU];
      Acc dhv[NU], hv[NU], hlv[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const size_t o = (size_t)(node + u * nrs) * F + p;
        sv[u] = sb[node + u * nrs];
        dhv[u] = v.L > 0 ? dH0[o] : (Acc)0;
        hv[u] = v.act == 0 ? H0[o] : (Acc)0;
        hlv[u] = HL[o];
      }
#pragma unroll
      for (int u = 0; u < NU; ++u) one(sv[u], dhv[u], hv[u], hlv[u]);
    }
    for (; node < v.n; node += nrs) {
      const size_t o = (size_t)node * F + p;
      one(sb[node], v.L > 0 ? dH0[o] : (Acc)0, v.act == 0 ? H0[o] : (Acc)0, HL[o]);
    }
    za += ca * z;
    zp += cp * z;
    ua += ca * nup;
    up += cp * nup;
    sca += ca;
    scp += cp;
  }
  __shared__ double red[4][256];
  __shared__ double red_up[2][256 / F];   // per row slot rs (the p == 0 threads)
  if (p == 0) {
    red_up[0][rs] = ua;
    red_up[1][rs] = up;
  }
  __shared__ double sdh[2][F];   // summed dH^0 per spin value, logical order
  red[0][threadIdx.x] = e0;
  red[1][threadIdx.x] = e1;
  red[2][threadIdx.x] = za;
  red[3][threadIdx.x] = zp;
  __syncthreads();
  double s0 = 0, s1 = 0, sa = 0, sp = 0;
  const int f = P::lc(p / NS, p % NS);
  if (threadIdx.x < F) {
    for (int r = 0; r < nrs; ++r) {
      s0 += red[0][r * F + p];
      s1 += red[1][r * F + p];
      sa += red[2][r * F + p];
      sp += red[3][r * F + p];
    }
    sdh[0][f] = s0;
    sdh[1][f] = s1;
  }
  __syncthreads();
  if (v.act != 0 && threadIdx.x < F) {
    // VJP of h = LN(ReLU(u)), u = W_e[x] + b_e, in FP64 from theta, for x = 0, 1
    const double* We = v.theta;
    const double* be = v.theta + 2 * F;
    double dx[2];
    for (int x = 0; x < 2; ++x) {
      double mu = 0.0, var = 0.0;
      for (int g = 0; g < F; ++g) mu += fmax(We[x * F + g] + be[g], 0.0);
      mu /= F;
      for (int g = 0; g < F; ++g) {
        const double d = fmax(We[x * F + g] + be[g], 0.0) - mu;
        var += d * d;
      }
      const double r = 1.0 / sqrt(var / F + kLnEps);
      double a = 0.0, b = 0.0;
      for (int g = 0; g < F; ++g) {
        const double hg = (fmax(We[x * F + g] + be[g], 0.0) - mu) * r;
        a += sdh[x][g];
        b += sdh[x][g] * hg;
      }
      const double u = We[x * F + f] + be[f];
      const double hf = (fmax(u, 0.0) - mu) * r;
      dx[x] = u > 0.0 ? r * (sdh[x][f] - a / F - hf * b / F) : 0.0;
    }
    s0 = dx[0];
    s1 = dx[1];
  }
  if (threadIdx.x < F) {
    const int nW = v.tied ? 1 : v.L;
    double* g = part + (size_t)blockIdx.x * v.npar;
    g[f] += s0;             // W_e[0][f]
    g[F + f] += s1;         // W_e[1][f]
    g[2 * F + f] += s0 + s1;  // b_e[f]
    double* gva = g + 3 * F + (size_t)nW * (2 * F * F + F);
    gva[f] += sa;
    gva[F + 3 + f] += sp;   // v_p
  }
  // one-hot counts and head biases: z[F] = #down, z[F+1] = #up
  if (threadIdx.x == 0) {
    double cup = 0, pup = 0;
    for (int r = 0; r < nrs; ++r) {
      cup += red_up[0][r];
      pup += red_up[1][r];
    }
    const int nW = v.tied ? 1 : v.L;
    double* gva = part + (size_t)blockIdx.x * v.npar + 3 * F + (size_t)nW * (2 * F * F + F);
    gva[F] += v.n * sca - cup;
    gva[F + 1] += cup;
    gva[F + 2] += sca;
    gva[F + 3 + F] += v.n * scp - pup;
    gva[F + 3 + F + 1] += pup;
    gva[F + 3 + F + 2] += scp;
  }
}

}  // namespace gna
