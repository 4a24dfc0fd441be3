// Incremental local energy: log psi(s^ij) - log psi(s) from the swapped sites'
// receptive field only.
//
// Exchanging the spins of bond (i, j) changes the layer-l embedding of exactly
// the nodes within graph distance l of {i, j} (the ball C_l), because layer l of
// Eq. 1 reads a node and its neighbours.  With the base planes of sample s
// (layer outputs H^l and message products G^l = H^l W_msg, written by the base
// pass), layer l is recomputed for the rows of C_l only:
//   G'_m = H'^{l-1}_m W_msg                  for m in C_l
//   P'_n = b + H'^{l-1}_n W_self + sum_d A_hat[n][d] G'^{l-1}_{nbr}   for n in C_l
// where H'^{l-1} equals the base rows outside C_{l-1}.  The rows are computed with
// the same instructions, operand order and reduction order as the full
// evaluation, so they are bit-identical to it, and
//   Delta = (v_a + i v_p) . sum_{n in C_L} (H'^L_n - H^L_n).
//
// Work decomposition.  One workgroup advances S exchanges of the same sample in
// lockstep, layer by layer.  The balls are nested: the node list of a bond is
// C_0, then the nodes at distance 1, 2, ... L, so C_l is a prefix of it.  Each
// exchange owns one LDS buffer with a row per list position:
//   - the layer's tiles (16 list positions each) take H'^{l-1} of their rows in
//     C_{l-1} from the registers of the previous layer (or base H^{l-1} for
//     positions beyond |C_{l-1}|), form both products, and write rows [0, |C_l|)
//     of the buffer with G^{l-1}; rows [|C_l|, |C_{l+1}|) receive base G^{l-1}
//     rows, so that the gather reads only LDS (the list runs to C_{L+1});
//   - the gather and the activation leave H'^l in the tile owner's registers.
// Tile (job w, tile t) is owned by wave (t * njobs + w) % waves at every layer,
// so a layer's outputs never cross waves, and a layer needs two barriers (the G
// rows complete before the gather; the gather done before the next G rows).
//
// The same ball evaluation serves the Metropolis sampler (Section 3): there each
// job belongs to its own chain, and the recomputed rows H'^l (C_l) and G'^{l-1}
// (C_{l-1}) are written into that chain's planes as they are produced.  Rows read
// later in the same evaluation are never among the rows written before them
// (layer l reads H^{l-1} outside C_{l-1} and G^{l-1} outside C_l).  A rejected
// proposal is followed by a restore job: the same ball for the unexchanged
// configuration, which rewrites the old rows bit for bit.
#pragma once

#include "gna_kernels.h"

namespace gna {

struct IncNet {
  int n, F, L, dmax;
  int r8;                  // node-list slots per bond (max |C_{L+1}| rounded up to 8)
  const int2* ball_meta;   // [ne] (first entry of bond e's table (multiple of 8), its length in 16-byte vectors)
  const int* ball_cnt;     // [ne][L+2] |C_l|, l = 0 .. L+1
  const uint16_t* ball_tab;   // per bond: r8 node ids of C_{L+1}, then |C_L| x dmax neighbour
                              // list positions, padded to a multiple of 8 entries
  const void* ell_val;     // [npad][dmax] A_hat in Acc precision
};

// LDS layout of the incremental kernels (byte offsets) and launch shape
struct IncGeo {
  int nw;           // waves per workgroup
  int S;            // jobs (exchanges) in flight per workgroup (<= kIncMaxSwaps)
  int row_elems;    // LDS row stride in Acc elements
  int rows;         // buffer rows per job (max |C_{L+1}|)
  int tabw;         // entries per job table in LDS (r8 + max|C_L| * dmax, multiple of 8)
  int spw;          // bytes per spin configuration in LDS
  int off_w, off_buf, off_tab, off_sp, off_red, off_bias, off_emb, off_head, off_ev, off_list, off_cpy;
  int off_edges;    // bond endpoints [n_edges] (int2) in LDS (the sweep kernel), or -1
  int xcd;          // items are grouped per XCD (blocks b with equal b % xcd share a sample)
  int lds_bytes;
};

constexpr int kIncMaxSwaps = 8;
constexpr int kIncCopy = 4;   // 16-byte base-row copies held in registers per thread

// job flags
constexpr int kJobSwap = 1;      // evaluate the exchanged configuration (else the current one)
constexpr int kJobReadout = 2;   // accumulate the readout difference

// The jobs of one group (LDS, written before the group's first barrier)
struct IncJobs {
  int cnt[kIncMaxSwaps][18];   // |C_l| of the job's bond
  int2 ij[kIncMaxSwaps];       // bond endpoints
  int e[kIncMaxSwaps];         // bond index
  int flags[kIncMaxSwaps];
  int spoff[kIncMaxSwaps];     // byte offset of the job's spins in the spin area
  long long pboff[kIncMaxSwaps];   // element offset of the job's planes
  int2 meta[kIncMaxSwaps];         // ball_meta of the job's bond
  int2 lay[17];                    // layer l: (first copy-list entry, copy rows) of the group
};

// LDS views of the incremental kernels
template <class P>
struct IncLds {
  typename P::WT* wl;
  typename P::Acc* buf;
  uint16_t* tab;
  int8_t* sp;
  double* red;                 // [kIncMaxSwaps][2][kMaxWaves]
  typename P::Acc* sbias;
  typename P::Acc* semb;
  double* shead;               // [2][F] readout weights v_a, v_p (FP64), slot order
  typename P::Acc* sev;
  int* slist;
  int4* cpy;                   // ring-row copy list of the group: (source offset lo, hi, LDS destination, 0)
  __device__ IncLds(const IncGeo& ig, unsigned char* smem) {
    using Acc = typename P::Acc;
    wl = reinterpret_cast<typename P::WT*>(smem + ig.off_w);
    buf = reinterpret_cast<Acc*>(smem + ig.off_buf);
    tab = reinterpret_cast<uint16_t*>(smem + ig.off_tab);
    sp = reinterpret_cast<int8_t*>(smem + ig.off_sp);
    red = reinterpret_cast<double*>(smem + ig.off_red);
    sbias = reinterpret_cast<Acc*>(smem + ig.off_bias);
    semb = reinterpret_cast<Acc*>(smem + ig.off_emb);
    shead = reinterpret_cast<double*>(smem + ig.off_head);
    sev = reinterpret_cast<Acc*>(smem + ig.off_ev);
    slist = reinterpret_cast<int*>(smem + ig.off_list);
    cpy = reinterpret_cast<int4*>(smem + ig.off_cpy);
  }
};

// weights (tied: one layer) and the small tables -> LDS
template <class P, int F>
__device__ void inc_stage(const Net& net, const IncNet& inc, const IncLds<P>& x) {
  using Acc = typename P::Acc;
  using WT = typename P::WT;
  constexpr int NS = F / 4;
  const int bd = blockDim.x;
  const WT* src = reinterpret_cast<const WT*>(net.wfrag);
  for (int k = threadIdx.x; k < P::WBLK * 2 * F * F; k += bd) x.wl[k] = src[k];
  for (int k = threadIdx.x; k < F; k += bd)
    x.sbias[k] = reinterpret_cast<const Acc*>(net.bias)[P::lc(k / NS, k % NS)];   // slot order
  for (int k = threadIdx.x; k < 2 * F; k += bd) x.semb[k] = reinterpret_cast<const Acc*>(net.emb)[k];
  for (int k = threadIdx.x; k < F; k += bd) {
    const int f = P::lc(k / NS, k % NS);
    x.shead[k] = net.head_a[f];
    x.shead[F + k] = net.head_p[f];
  }
  const Acc* ev = reinterpret_cast<const Acc*>(inc.ell_val);
  for (int k = threadIdx.x; k < net.n * inc.dmax; k += bd) x.sev[k] = ev[k];
}

// One group of nsw jobs: tables -> LDS, then layers 1..L over the jobs' balls.
// Entry: jobs.{ij, e, flags, spoff, pboff, meta, cnt} written and visible (after a barrier).
// Exit: readout partials of job j in red[(2j + {0,1}) * kMaxWaves + wave] for jobs
// with kJobReadout (the caller synchronises before reading them).  With WRITE the
// recomputed rows are stored into the jobs' planes.
template <class P, int F, int MAXT, bool WRITE, int NCOPY = kIncCopy, int GU = 4>
__device__ void inc_group(const Net& net, const IncNet& inc, const IncGeo& ig, const IncLds<P>& x, IncJobs& jobs,
                          int nsw, typename P::Acc* planes, unsigned char* smem) {
  using Acc = typename P::Acc;
  using CF = typename P::CF;
  constexpr int NS = F / 4, MT = F / 16, KSB = F / P::KS, VEC = P::VEC;
  constexpr int SM = kIncMaxSwaps;
  constexpr int VPR = F * (int)sizeof(Acc) / 16;   // 16-byte vectors per row
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q = lane >> 4, col = lane & 15;
  const int nw = ig.nw, Lr = net.L, dm = inc.dmax, bd = blockDim.x;
  nsw = __builtin_amdgcn_readfirstlane(nsw);   // the same in every thread: scalar branches
  const size_t plane = (size_t)net.g.npad * F;
  const Acc* bias = x.sbias + q * NS;

  // tables of the group -> LDS (16-byte vectors)
  {
    const int tv = ig.tabw / 8;
    for (int k = threadIdx.x; k < nsw * tv; k += bd) {
      const int w = k / tv, v = k % tv;
      const int2 mt = jobs.meta[w];
      if (v < mt.y) reinterpret_cast<int4*>(x.tab + w * ig.tabw)[v] = reinterpret_cast<const int4*>(inc.ball_tab + mt.x)[v];
    }
  }
  // copy list: the rows of ring l+1 (list positions [|C_l|, |C_{l+1}|)) of every job, for
  // layers l = 1..L in turn, with their source offset (node row of the job's planes) and
  // LDS destination; entry of (job w, position rr) at layer l:
  //   sum_w' (|C_l|_w' - |C_1|_w') + sum_{w' < w} (|C_{l+1}|_w' - |C_l|_w') + rr - |C_l|_w
  {
    int tot = 0;
    for (int w = 0; w < nsw; ++w) tot += jobs.cnt[w][Lr + 1] - jobs.cnt[w][1];
    for (int k = threadIdx.x; k < tot; k += bd) {
      int w = 0, start = 0;
      while (k - start >= jobs.cnt[w][Lr + 1] - jobs.cnt[w][1]) {
        start += jobs.cnt[w][Lr + 1] - jobs.cnt[w][1];
        ++w;
      }
      const int rr = jobs.cnt[w][1] + (k - start);
      int l = 1;
      while (rr >= jobs.cnt[w][l + 1]) ++l;
      int idx = rr - jobs.cnt[w][l];
      for (int u = 0; u < nsw; ++u) {
        idx += jobs.cnt[u][l] - jobs.cnt[u][1];
        if (u < w) idx += jobs.cnt[u][l + 1] - jobs.cnt[u][l];
      }
      const int nd = inc.ball_tab[jobs.meta[w].x + rr];
      const long long so = jobs.pboff[w] + (long long)nd * F;
      x.cpy[idx] = make_int4((int)(unsigned)so, (int)(so >> 32),
                             ig.off_buf + (w * ig.rows + rr) * ig.row_elems * (int)sizeof(Acc), 0);
    }
    if ((int)threadIdx.x <= Lr) {
      const int l = threadIdx.x;
      int base = 0, rows = 0;
      for (int u = 0; u < nsw; ++u) {
        base += jobs.cnt[u][max(l, 1)] - jobs.cnt[u][1];
        rows += l >= 1 ? jobs.cnt[u][l + 1] - jobs.cnt[u][l] : 0;
      }
      jobs.lay[l] = make_int2(base, rows);
    }
  }
  __syncthreads();
  // spin of node nd in the configuration job w evaluates
  auto xspin = [&](int w, int nd) {
    const int8_t* spw = x.sp + jobs.spoff[w];
    const int2 ij = jobs.ij[w];
    int8_t v = spw[nd];
    if (jobs.flags[w] & kJobSwap) v = (nd == ij.x) ? spw[ij.y] : ((nd == ij.y) ? spw[ij.x] : v);
    return v > 0 ? 1 : 0;
  };
  // layer inputs of this wave's tiles: a tile belongs to the same wave at every
  // layer, so H'^l of its rows in C_l stays in registers as the next layer's input.
  // The lanes of its rows in ring l+1 (list positions [|C_l|, |C_{l+1}|)) take the
  // base H^l rows instead: they are read into those lanes of hn right after the
  // tile's layer-l activation, so that they arrive during the rest of the layer
  // (no layer of the group writes them).
  Acc hn[MAXT][NS];
  auto prefetch_in = [&](int k, int l) {   // l >= 2: base H^{l-1} of ring l in tile k
    const int g = wv + k * nw;
    const int w = g % nsw, tt = g / nsw;
    const int cl = __builtin_amdgcn_readfirstlane(jobs.cnt[w][l]);
    const int cp = __builtin_amdgcn_readfirstlane(jobs.cnt[w][l - 1]);
    const int r = tt * 16 + col;
    if (tt * 16 < cl && r >= cp && r < cl) {
      const int nd = (int)x.tab[w * ig.tabw + r];
      gmem_read<Acc, NS>(planes + jobs.pboff[w] + (size_t)(l - 2) * plane + (size_t)nd * F + q * NS, hn[k]);
    }
  };
  for (int l = 1; l <= Lr; ++l) {
    // ---- base G^{l-1} rows of the nodes at distance l+1 -> buffer (requested first,
    // stored after this wave's products)
    using V4 = unsigned int __attribute__((ext_vector_type(4)));
    V4 cvv[NCOPY];
    int cdst[NCOPY];
    {
      const int2 lay = make_int2(__builtin_amdgcn_readfirstlane(jobs.lay[l].x),
                                 __builtin_amdgcn_readfirstlane(jobs.lay[l].y));
      const int ctot = lay.y * VPR;
      const Acc* Gl = planes + (size_t)(Lr + l - 1) * plane;
      // copy item idx -> (source vector, byte offset of the destination in LDS)
      auto locate = [&](int idx, const V4*& src) {
        const int4 c = x.cpy[lay.x + idx / VPR];
        const int v = idx % VPR;
        const long long so = (long long)(((unsigned long long)(unsigned)c.y << 32) | (unsigned)c.x);
        src = reinterpret_cast<const V4*>(Gl + so) + v;
        return c.z + 16 * v;
      };
      const V4* ph = reinterpret_cast<const V4*>(planes + jobs.pboff[0]);   // in-bounds placeholder
#pragma unroll
      for (int u = 0; u < NCOPY; ++u) {   // no branches: the lookups overlap
        const int idx = threadIdx.x + u * bd;
        const V4* src = ph;
        const int o = locate(min(idx, max(ctot - 1, 0)), src);
        cdst[u] = idx < ctot ? o : -1;
        if (ctot == 0) src = ph;
        cvv[u] = *src;   // unconditional, so the value stays in registers
      }
      for (int idx = threadIdx.x + NCOPY * bd; idx < ctot; idx += bd) {   // rare: large rings
        const V4* src;
        const int o = locate(idx, src);
        *reinterpret_cast<V4*>(smem + o) = *src;
      }
    }
    // ---- this wave's tiles: job, row, |C_l|, |C_{l-1}| and node of each (looked up once)
    int trow[MAXT], tsw[MAXT], tcl[MAXT], tcp[MAXT], tnd[MAXT];
    bool tok[MAXT];
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      const int g = wv + k * nw;
      const int w = g % nsw, tt = g / nsw;
      tsw[k] = w;
      tcl[k] = __builtin_amdgcn_readfirstlane(jobs.cnt[w][l]);   // per job: uniform in the wave
      tcp[k] = __builtin_amdgcn_readfirstlane(jobs.cnt[w][l - 1]);
      tok[k] = tt * 16 < tcl[k];
      trow[k] = tt * 16 + col;
      tnd[k] = trow[k] < tcl[k] ? (int)x.tab[w * ig.tabw + trow[k]] : -1;
    }
    // ---- products: self -> registers, message -> buffer rows [0, |C_l|) in place
    // layer input of tile k: embedding (l = 1), else hn (H'^{l-1} of the previous
    // layer on C_{l-1}, the prefetched base H^{l-1} on ring l); zero past |C_l|
    auto load_in = [&](int k, Acc (&h)[NS]) {
      const int w = tsw[k], nd = tnd[k];
      if (l == 1) {
        const int xs = nd >= 0 ? xspin(w, nd) : 0;
#pragma unroll
        for (int i = 0; i < NS; ++i) h[i] = nd >= 0 ? x.semb[xs * F + P::lc(q, i)] : (Acc)0;
      } else {
#pragma unroll
        for (int i = 0; i < NS; ++i) h[i] = nd >= 0 ? hn[k][i] : (Acc)0;
      }
    };
    CF acc[MAXT][MT];
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      if (!tok[k]) continue;
      const int w = tsw[k], r = trow[k];
      const int cl = tcl[k], cp = tcp[k];
      const int nd = tnd[k];
      Acc* pw = planes + jobs.pboff[w];
      Acc h[NS];
      load_in(k, h);
      Acc* row = x.buf + ((size_t)w * ig.rows + r) * ig.row_elems + q * NS;
      auto afr = [&](int blk, int st, int t) { return x.wl + (((blk * KSB + st) * MT + t) * 64 + lane) * VEC; };
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        CF a, gs = CF{0, 0, 0, 0};
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) a[rr] = bias[4 * t + rr];
#pragma unroll
        for (int st = 0; st < KSB; ++st) {
          const auto bop = P::make_b(&h[st * VEC]);
          gs = P::mma(P::load_a(afr(0, st, t)), bop, gs);
          a = P::mma(P::load_a(afr(1, st, t)), bop, a);
        }
        acc[k][t] = a;
        Acc gm[4] = {gs[0], gs[1], gs[2], gs[3]};
        if (r < cl) lds_write<Acc, 4>(row + 4 * t, gm);
        if (WRITE && r < cp)   // G^{l-1} changed on C_{l-1}
          lds_write<Acc, 4>(pw + (size_t)(Lr + l - 1) * plane + (size_t)nd * F + q * NS + 4 * t, gm);
        if (GU < 4) __builtin_amdgcn_sched_barrier(0);   // low-register shape: one output tile at a time
      }
    }
#pragma unroll
    for (int u = 0; u < NCOPY; ++u)
      if (cdst[u] >= 0) *reinterpret_cast<V4*>(smem + cdst[u]) = cvv[u];
    __syncthreads();   // every G^{l-1} row of every job is in its buffer
    // ---- gather, activation; readout difference at the last layer
    if (l == Lr && lane == 0)
      for (int w = 0; w < nsw; ++w) x.red[(2 * w) * kMaxWaves + wv] = x.red[(2 * w + 1) * kMaxWaves + wv] = 0.0;
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      if (!tok[k]) {
        if (l < Lr) prefetch_in(k, l + 1);   // a tile that starts at the next layer
        continue;
      }
      const int w = tsw[k], r = trow[k];
      const uint16_t* tw = x.tab + w * ig.tabw;
      const int nd = tnd[k];
      const Acc* bw = x.buf + (size_t)w * ig.rows * ig.row_elems;
      Acc* pw = planes + jobs.pboff[w];
      const bool last = l == Lr;
      const bool rd = last && (jobs.flags[w] & kJobReadout);
      double r0[2] = {0.0, 0.0};   // base readout partials of the node (FP64)
      if (rd && nd >= 0) {
        const double* rp = reinterpret_cast<const double*>(pw + (size_t)(Lr - 1) * plane) + (size_t)nd * 8 + q * 2;
        r0[0] = rp[0];
        r0[1] = rp[1];
      }
      Acc m[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) m[i] = (Acc)0;
      if (nd >= 0) {
        const uint16_t* nbp = tw + inc.r8 + r * dm;
        for (int d = 0; d < dm; d += 4) {
          const uint2 pv = *reinterpret_cast<const uint2*>(nbp + d);
          const int pc[4] = {(int)(pv.x & 0xffffu), (int)(pv.x >> 16), (int)(pv.y & 0xffffu), (int)(pv.y >> 16)};
          const Acc* wp = x.sev + nd * dm + d;
          const Acc wt[4] = {wp[0], wp[1], wp[2], wp[3]};
#pragma unroll
          for (int u = 0; u < 4; u += GU) {
#pragma unroll
           for (int uu = u; uu < u + GU; ++uu) {
            Acc rowv[NS];
            lds_read<Acc, NS>(bw + pc[uu] * ig.row_elems + q * NS, rowv);
#pragma unroll
            for (int i = 0; i < NS; ++i) m[i] += wt[uu] * rowv[i];
           }
           if (GU < 4) __builtin_amdgcn_sched_barrier(0);   // keep GU rows in flight at most
          }
        }
      }
      if (net.act == 0) {
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) hn[k][4 * t + rr] = P::act(acc[k][t][rr] + m[4 * t + rr]);
      } else {   // the four lanes of a row are active together (tok is wave-uniform)
        Acc pre[NS], y[NS];
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) pre[4 * t + rr] = acc[k][t][rr] + m[4 * t + rr];
        relu_ln_row<Acc, NS>(pre, y, hn[k]);
      }
      if (last && (rd || WRITE)) {   // wave-uniform
        // FP64 readout partials of this node, formed as in the full evaluation
        const double* va = x.shead + q * NS;
        const double* vp = x.shead + F + q * NS;
        double ta1 = 0, tp1 = 0;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          ta1 += va[i] * (double)hn[k][i];
          tp1 += vp[i] * (double)hn[k][i];
        }
        if (rd) {
          double pa = nd >= 0 ? ta1 - r0[0] : 0.0;
          double pp = nd >= 0 ? tp1 - r0[1] : 0.0;
          pa = wave_sum_dpp(pa);
          pp = wave_sum_dpp(pp);
          if (lane == 0) {
            x.red[(2 * w) * kMaxWaves + wv] += pa;
            x.red[(2 * w + 1) * kMaxWaves + wv] += pp;
          }
        }
        if (WRITE && nd >= 0) {   // after the base partials were read
          const double rv[2] = {ta1, tp1};
          lds_write<double, 2>(reinterpret_cast<double*>(pw + (size_t)(Lr - 1) * plane) + (size_t)nd * 8 + q * 2, rv);
        }
      } else if (WRITE && !last && nd >= 0) {   // H^l changed on C_l
        lds_write<Acc, NS>(pw + (size_t)(l - 1) * plane + (size_t)nd * F + q * NS, hn[k]);
      }
      if (l < Lr) prefetch_in(k, l + 1);   // after the rows' own values were used
    }
    if (l < Lr) __syncthreads();   // every gather read of the buffers is done before new G rows
  }
}

// compensated sum step (Neumaier)
__device__ __forceinline__ void inc_neumaier(double& s, double& c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

// Local energy: the exchanges of the anti-aligned bonds of every sample.
template <class P, int F, int MAXT, int NT>
__global__ __launch_bounds__(NT) void k_eloc_inc(Net net, IncNet inc, IncGeo ig, const int8_t* __restrict__ spins,
                                                  int B, const typename P::Acc* __restrict__ planes, int n_chunks,
                                                  int chunk, double* __restrict__ partial, int* __restrict__ cnt) {
  using Acc = typename P::Acc;
  constexpr int SM = kIncMaxSwaps;
  extern __shared__ __align__(16) unsigned char smem[];
  IncLds<P> x(ig, smem);
  __shared__ IncJobs jobs;
  __shared__ int s_wc[kMaxWaves];
  __shared__ double s_acc[SM][4];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = ig.nw, Lr = net.L, S = ig.S, bd = blockDim.x;
  const size_t plane = (size_t)net.g.npad * F;
  Acc* pl = const_cast<Acc*>(planes);   // read only: inc_group without WRITE
  inc_stage<P, F>(net, inc, x);
  __syncthreads();

  // XCD-aware order: the blocks of one XCD (equal blockIdx % xcd) walk the chunks of
  // the same samples together, so a sample's base planes stay in that XCD's L2
  const int X = ig.xcd;
  const int per_x = gridDim.x / X;
  const int xid = blockIdx.x % X, slot = blockIdx.x / X;
  const long long per_xcd_items = (long long)((B - xid + X - 1) / X) * n_chunks;
  for (long long jj = slot; jj < per_xcd_items; jj += per_x) {
    const int b = xid + X * (int)(jj / n_chunks), c = (int)(jj % n_chunks);
    const int it = b * n_chunks + c;
    for (int k = threadIdx.x; k < net.n; k += bd) x.sp[k] = spins[(size_t)b * net.n + k];
    __syncthreads();
    // anti-aligned bonds of the chunk, in bond order (ballot compaction)
    const int e0 = c * chunk, clen = max(0, min(net.ne, e0 + chunk) - e0);
    int nanti = 0;
    {
      int flag = 0;
      if ((int)threadIdx.x < clen) {
        const int2 ij = net.edges[e0 + threadIdx.x];
        flag = x.sp[ij.x] != x.sp[ij.y];
      }
      const unsigned long long m = __ballot(flag);
      if (lane == 0) s_wc[wv] = __popcll(m);
      __syncthreads();
      int before = 0;
      for (int v = 0; v < nw; ++v) {
        const int cv = s_wc[v];
        if (v < wv) before += cv;
        nanti += cv;
      }
      if (flag) x.slist[before + __popcll(m & ((1ull << lane) - 1ull))] = e0 + threadIdx.x;
    }
    // per-job-slot compensated sums in LDS (thread w accumulates slot w)
    if ((int)threadIdx.x < SM)
      s_acc[threadIdx.x][0] = s_acc[threadIdx.x][1] = s_acc[threadIdx.x][2] = s_acc[threadIdx.x][3] = 0.0;
    for (int g0 = 0; g0 < nanti; g0 += S) {
      const int nsw = min(S, nanti - g0);
      __syncthreads();   // slist visible; the previous group is done with the job tables
      if ((int)threadIdx.x < nsw) {
        const int w = threadIdx.x, eg = x.slist[g0 + w];
        jobs.e[w] = eg;
        jobs.ij[w] = net.edges[eg];
        jobs.meta[w] = inc.ball_meta[eg];
        for (int l = 0; l < Lr + 2; ++l) jobs.cnt[w][l] = inc.ball_cnt[eg * (Lr + 2) + l];
        jobs.flags[w] = kJobSwap | kJobReadout;
        jobs.spoff[w] = 0;
        jobs.pboff[w] = (long long)b * 2 * Lr * plane;
      }
      __syncthreads();
      inc_group<P, F, MAXT, false, NT == 1024 ? 1 : kIncCopy, NT == 1024 ? 1 : 4>(net, inc, ig, x, jobs, nsw, pl, smem);
      __syncthreads();   // readout partials of every wave
      if ((int)threadIdx.x < nsw) {
        const int w = threadIdx.x;
        double da = 0.0, dp = 0.0;
        for (int v = 0; v < nw; ++v) {
          da += x.red[(2 * w) * kMaxWaves + v];
          dp += x.red[(2 * w + 1) * kMaxWaves + v];
        }
        const double mm = exp(da);
        double sn, cs;
        sincos(dp, &sn, &cs);
        inc_neumaier(s_acc[w][0], s_acc[w][1], mm * cs);
        inc_neumaier(s_acc[w][2], s_acc[w][3], mm * sn);
      }
    }
    // combine the slots in slot order
    __syncthreads();
    if (threadIdx.x == 0) {
      double tr = 0, tcr = 0, ti = 0, tci = 0;
      for (int w = 0; w < min(S, SM); ++w) {
        inc_neumaier(tr, tcr, s_acc[w][0]);
        tcr += s_acc[w][1];
        inc_neumaier(ti, tci, s_acc[w][2]);
        tci += s_acc[w][3];
      }
      double* o = partial + 4 * (size_t)it;
      o[0] = tr; o[1] = tcr; o[2] = ti; o[3] = tci;
      cnt[it] = nanti;
    }
    __syncthreads();
  }
}

// Metropolis spin-swap sweeps (Section 3) with incremental proposals.  Slot w of
// block x runs chains x + (w + S k) * gridDim.x one after the other; the draws are
// the ones of the full-recompute sampler (Philox4x32-10, counter (step, chain, 0),
// key = seed), and a proposal is accepted when u < exp(2 Re Delta).  The chains'
// planes must hold their current configurations (base pass) and are kept current.
// log psi is not tracked here: the caller evaluates the final configurations.
template <class P, int F, int MAXT, int NT>
__global__ __launch_bounds__(NT) void k_sweep_inc(Net net, IncNet inc, IncGeo ig, int8_t* __restrict__ spins,
                                                   typename P::Acc* planes, int B, int n_sweeps,
                                                   unsigned long long seed, unsigned long long counter_base,
                                                   const unsigned long long* __restrict__ counter_dev,
                                                   int* __restrict__ n_accept) {
  constexpr int SM = kIncMaxSwaps;
  extern __shared__ __align__(16) unsigned char smem[];
  IncLds<P> x(ig, smem);
  __shared__ IncJobs jobs;
  __shared__ int s_chain[SM], s_acc[SM], s_prop[SM], s_pend[SM], s_job[SM], s_done[SM], s_jslot[SM];
  __shared__ long long s_t[SM];
  __shared__ double s_u[SM];
  __shared__ int s_nsw, s_switch;
  const int nw = ig.nw, S = ig.S, bd = blockDim.x;
  const size_t per_chain = (size_t)2 * net.L * net.g.npad * F;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const long long total = (long long)n_sweeps * net.n;
  if (counter_dev) counter_base += *counter_dev;   // graph replays read the current base
  inc_stage<P, F>(net, inc, x);
  // bond endpoints in LDS when they fit: the proposal draws look them up one after another
  const int2* edges = net.edges;
  if (ig.off_edges >= 0) {
    int2* se = reinterpret_cast<int2*>(smem + ig.off_edges);
    for (int k = threadIdx.x; k < net.ne; k += bd) se[k] = net.edges[k];
    edges = se;
  }
  if ((int)threadIdx.x < S) {
    const int w = threadIdx.x;
    const int b = blockIdx.x + w * gridDim.x;
    s_chain[w] = b < B ? b : -1;
    s_t[w] = 0;
    s_acc[w] = 0;
    s_pend[w] = -1;
  }
  __syncthreads();
  for (int w = 0; w < S; ++w)
    if (s_chain[w] >= 0)
      for (int k = threadIdx.x; k < net.n; k += bd) x.sp[w * ig.spw + k] = spins[(size_t)s_chain[w] * net.n + k];
  while (true) {
    __syncthreads();
    // each slot's next job: a pending restore, else its next anti-aligned proposal
    if ((int)threadIdx.x < S) {
      const int w = threadIdx.x, b = s_chain[w];
      int job = 0;   // 0 none, 1 proposal, 2 restore
      s_done[w] = 0;
      if (b >= 0) {
        if (s_pend[w] >= 0) {
          job = 2;
        } else {
          const int8_t* spw = x.sp + w * ig.spw;
          long long t = s_t[w];
          while (t < total) {
            const unsigned long long step = counter_base + (unsigned long long)t;
            uint32_t c[4] = {(uint32_t)step, (uint32_t)(step >> 32), (uint32_t)b, 0u};
            philox4x32_10(c, k0, k1);
            const int e = (int)(((unsigned long long)c[0] * (unsigned long long)net.ne) >> 32);
            const int2 ij = edges[e];
            if (spw[ij.x] != spw[ij.y]) {
              s_prop[w] = e;   // the proposal's bond
              s_u[w] = ((double)c[1] + 0.5) * 2.3283064365386963e-10;   // 2^-32
              job = 1;
              break;
            }
            ++t;   // identity step
          }
          s_t[w] = t;
          if (!job) s_done[w] = 1;
        }
      }
      s_job[w] = job;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int sw = 0, k = 0;
      for (int w = 0; w < S; ++w) {
        sw |= s_done[w];
        if (s_job[w]) s_jslot[k++] = w;
      }
      s_switch = sw;
      s_nsw = k;
    }
    __syncthreads();
    if (s_switch) {
      // finished chains: spins and acceptance count out, the slot's next chain in
      for (int w = 0; w < S; ++w) {
        if (!s_done[w]) continue;
        const int b = s_chain[w];
        for (int k = threadIdx.x; k < net.n; k += bd) spins[(size_t)b * net.n + k] = x.sp[w * ig.spw + k];
        const int nb = b + S * gridDim.x;
        if (nb < B)
          for (int k = threadIdx.x; k < net.n; k += bd) x.sp[w * ig.spw + k] = spins[(size_t)nb * net.n + k];
      }
      __syncthreads();
      if ((int)threadIdx.x < S && s_done[threadIdx.x]) {
        const int w = threadIdx.x, b = s_chain[w];
        if (n_accept) n_accept[b] = s_acc[w];
        const int nb = b + S * gridDim.x;
        s_chain[w] = nb < B ? nb : -1;
        s_t[w] = 0;
        s_acc[w] = 0;
        s_pend[w] = -1;
      }
      continue;   // select again (a slot's proposal is drawn again: its t is unchanged)
    }
    const int nsw = s_nsw;
    if (nsw == 0) break;
    if ((int)threadIdx.x < nsw) {
      const int j = threadIdx.x, w = s_jslot[j];
      const int e = s_job[w] == 1 ? s_prop[w] : s_pend[w];
      jobs.e[j] = e;
      jobs.ij[j] = edges[e];
      jobs.meta[j] = inc.ball_meta[e];
      for (int l = 0; l < net.L + 2; ++l) jobs.cnt[j][l] = inc.ball_cnt[e * (net.L + 2) + l];
      jobs.flags[j] = s_job[w] == 1 ? (kJobSwap | kJobReadout) : 0;
      jobs.spoff[j] = w * ig.spw;
      jobs.pboff[j] = (long long)s_chain[w] * (long long)per_chain;
    }
    __syncthreads();
    inc_group<P, F, MAXT, true, NT == 1024 ? 1 : kIncCopy, NT == 1024 ? 1 : 4>(net, inc, ig, x, jobs, nsw, planes, smem);
    __syncthreads();   // readout partials of every wave
    if ((int)threadIdx.x < nsw) {
      const int j = threadIdx.x, w = s_jslot[j];
      if (s_job[w] == 1) {
        double da = 0.0;
        for (int v = 0; v < nw; ++v) da += x.red[(2 * j) * kMaxWaves + v];
        if (s_u[w] < exp(2.0 * da)) {   // accept: the planes already hold the new rows
          int8_t* spw = x.sp + w * ig.spw;
          const int2 ij = jobs.ij[j];
          const int8_t tmp = spw[ij.x];
          spw[ij.x] = spw[ij.y];
          spw[ij.y] = tmp;
          ++s_acc[w];
        } else {
          s_pend[w] = s_prop[w];   // reject: the restore job of this bond comes next
        }
        ++s_t[w];
      } else {
        s_pend[w] = -1;   // restored
      }
    }
  }
}

// Base pass: the full evaluation of every sample, keeping its planes.
template <class P, int F, int TPW, int NCH>
__global__ __launch_bounds__(512) void k_inc_base(Net net, const int8_t* __restrict__ spins, int B,
                                                  typename P::Acc* planes, double* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  Smem<P> s(net.g, smem);
  stage_graph<P>(net, s);
  if (net.tied) stage_weights<P, F>(net, s, 0);
  __syncthreads();
  const size_t per = (size_t)2 * net.L * net.g.npad * F;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    load_spins<P>(net, s, spins + (size_t)b * net.n);
    double la = 0, ph = 0;
    eval_config<P, F, TPW, NCH, 2>(net, s, -1, -1, la, ph, planes + b * per);
    if (out && threadIdx.x == 0) {
      out[2 * (size_t)b] = la;
      out[2 * (size_t)b + 1] = ph;
    }
  }
}

}  // namespace gna
