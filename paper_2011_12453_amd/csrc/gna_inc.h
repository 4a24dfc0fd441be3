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
//   - at the start of layer l, rows [0, |C_{l-1}|) hold H'^{l-1};
//   - the layer's tiles (16 list positions each) read those rows (or base H^{l-1}
//     for positions beyond |C_{l-1}|), form both products, and overwrite rows
//     [0, |C_l|) with G^{l-1} in place; rows [|C_l|, |C_{l+1}|) receive base
//     G^{l-1} rows, so that the gather reads only LDS (the list runs to C_{L+1});
//   - after the gather, rows [0, |C_l|) receive H'^l.
// Tile (swap w, tile t) is owned by wave (t * nswap + w) % waves at every layer,
// so a wave reads back only rows it wrote itself and a layer needs two barriers.
#pragma once

#include "gna_kernels.h"

namespace gna {

struct IncNet {
  int n, F, L, dmax;
  int r4;                  // node-list slots per bond (max |C_{L+1}| rounded up to 4)
  const int* ball_off;     // [ne] first int of bond e's table (multiple of 4)
  const int* ball_cnt;     // [ne][L+2] |C_l|, l = 0 .. L+1
  const int* ball_tab;     // per bond: r4 node ids of C_{L+1} (-1 padded), then |C_L| x dmax
                           // neighbour list positions; 4-int aligned
  const void* ell_val;     // [npad][dmax] A_hat in Acc precision
};

// LDS layout of k_eloc_inc (byte offsets) and launch shape
struct IncGeo {
  int nw;           // waves per workgroup
  int S;            // exchanges in flight per workgroup (<= kIncMaxSwaps)
  int row_elems;    // LDS row stride in Acc elements
  int rows;         // buffer rows per exchange (max |C_{L+1}|)
  int tabw;         // ints per exchange table in LDS (r4 + rows * dmax, multiple of 4)
  int off_w, off_buf, off_tab, off_sp, off_red, off_bias, off_emb, off_head, off_ev, off_list;
  int xcd;          // items are grouped per XCD (blocks b with equal b % xcd share a sample)
  int lds_bytes;
};

constexpr int kIncMaxSwaps = 8;
constexpr int kIncCopy = 4;   // 16-byte base-row copies held in registers per thread

template <class P, int F, int MAXT>
__global__ __launch_bounds__(512) void k_eloc_inc(Net net, IncNet inc, IncGeo ig, const int8_t* __restrict__ spins,
                                                  int B, const typename P::Acc* __restrict__ planes, int n_chunks,
                                                  int chunk, double* __restrict__ partial, int* __restrict__ cnt) {
  using Acc = typename P::Acc;
  using WT = typename P::WT;
  using CF = typename P::CF;
  constexpr int NS = F / 4, MT = F / 16, KSB = F / P::KS, VEC = P::VEC;
  constexpr int SM = kIncMaxSwaps;
  constexpr int VPR = F * (int)sizeof(Acc) / 16;   // 16-byte vectors per row
  extern __shared__ __align__(16) unsigned char smem[];
  WT* wl = reinterpret_cast<WT*>(smem + ig.off_w);
  Acc* buf = reinterpret_cast<Acc*>(smem + ig.off_buf);
  int* tab = reinterpret_cast<int*>(smem + ig.off_tab);
  int8_t* sp = reinterpret_cast<int8_t*>(smem + ig.off_sp);
  double* red = reinterpret_cast<double*>(smem + ig.off_red);   // [SM][2][kMaxWaves]
  Acc* sbias = reinterpret_cast<Acc*>(smem + ig.off_bias);
  Acc* semb = reinterpret_cast<Acc*>(smem + ig.off_emb);
  double* shead = reinterpret_cast<double*>(smem + ig.off_head);
  Acc* sev = reinterpret_cast<Acc*>(smem + ig.off_ev);
  int* slist = reinterpret_cast<int*>(smem + ig.off_list);       // anti-aligned bonds of the item
  __shared__ int s_cnt[SM][18];
  __shared__ int2 s_ij[SM];
  __shared__ int s_wc[kMaxWaves];
  __shared__ double s_acc[SM][4];

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q = lane >> 4, col = lane & 15;
  const int nw = ig.nw, Lr = net.L, dm = inc.dmax, S = ig.S;
  const int bd = blockDim.x;
  const size_t plane = (size_t)net.g.npad * F;

  // stage weights (tied: one layer) and the small tables
  {
    const int nwt = 2 * F * F;
    const WT* src = reinterpret_cast<const WT*>(net.wfrag);
    for (int k = threadIdx.x; k < nwt; k += bd) wl[k] = src[k];
    for (int k = threadIdx.x; k < F; k += bd)
      sbias[k] = reinterpret_cast<const Acc*>(net.bias)[P::lc(k / NS, k % NS)];   // slot order
    for (int k = threadIdx.x; k < 2 * F; k += bd) semb[k] = reinterpret_cast<const Acc*>(net.emb)[k];
    for (int k = threadIdx.x; k < F + 3; k += bd) {
      shead[k] = net.head_a[k];
      shead[F + 3 + k] = net.head_p[k];
    }
    const Acc* ev = reinterpret_cast<const Acc*>(inc.ell_val);
    for (int k = threadIdx.x; k < net.n * dm; k += bd) sev[k] = ev[k];
  }
  __syncthreads();
  auto afrag = [&](int blk, int st, int t) { return wl + (((blk * KSB + st) * MT + t) * 64 + lane) * VEC; };
  const Acc* bias = sbias + q * NS;

  // XCD-aware order: the blocks of one XCD (equal blockIdx % xcd) walk the chunks of
  // the same samples together, so a sample's base planes stay in that XCD's L2
  const int X = ig.xcd;
  const int per_x = gridDim.x / X;
  const int xid = blockIdx.x % X, slot = blockIdx.x / X;
  const long long per_xcd_items = (long long)((B - xid + X - 1) / X) * n_chunks;
  for (long long jj = slot; jj < per_xcd_items; jj += per_x) {
    const int b = xid + X * (int)(jj / n_chunks), c = (int)(jj % n_chunks);
    const int it = b * n_chunks + c;
    for (int k = threadIdx.x; k < net.n; k += bd) sp[k] = spins[(size_t)b * net.n + k];
    __syncthreads();
    const Acc* pb = planes + (size_t)b * 2 * Lr * plane;
    // anti-aligned bonds of the chunk, in bond order (ballot compaction)
    const int e0 = c * chunk, clen = max(0, min(net.ne, e0 + chunk) - e0);
    int nanti = 0;
    {
      int flag = 0;
      if ((int)threadIdx.x < clen) {
        const int2 ij = net.edges[e0 + threadIdx.x];
        flag = sp[ij.x] != sp[ij.y];
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
      if (flag) slist[before + __popcll(m & ((1ull << lane) - 1ull))] = e0 + threadIdx.x;
    }
    // per-swap-slot compensated sums (thread w accumulates slot w)
    double sr = 0, cr = 0, si = 0, ci = 0;
    for (int g0 = 0; g0 < nanti; g0 += S) {
      const int nsw = min(S, nanti - g0);
      __syncthreads();   // slist visible; the previous group is done with tab / red
      // tables of the group -> LDS (16-byte vectors)
      {
        for (int k = threadIdx.x; k < nsw * (Lr + 2); k += bd) {
          const int w = k / (Lr + 2), l = k % (Lr + 2);
          s_cnt[w][l] = inc.ball_cnt[slist[g0 + w] * (Lr + 2) + l];
        }
        if ((int)threadIdx.x < nsw) s_ij[threadIdx.x] = net.edges[slist[g0 + threadIdx.x]];
        const int tv = ig.tabw / 4;
        for (int k = threadIdx.x; k < nsw * tv; k += bd) {
          const int w = k / tv, v = k % tv;
          const int eg = slist[g0 + w];
          const int nr = inc.ball_cnt[eg * (Lr + 2) + Lr];
          const int nv = (inc.r4 + nr * dm) / 4;   // this bond's table, in vectors
          if (v < nv)
            reinterpret_cast<int4*>(tab + w * ig.tabw)[v] =
                reinterpret_cast<const int4*>(inc.ball_tab + inc.ball_off[eg])[v];
        }
      }
      __syncthreads();
      // the exchanged configuration of swap w: spin of node nd
      auto xnew = [&](int w, int nd) {
        const int2 ij = s_ij[w];
        const int8_t v = (nd == ij.x) ? sp[ij.y] : ((nd == ij.y) ? sp[ij.x] : sp[nd]);
        return v > 0 ? 1 : 0;
      };
      for (int l = 1; l <= Lr; ++l) {
        const Acc* Hbase = pb + (size_t)(l - 2) * plane;           // H^{l-1} (l >= 2)
        const Acc* Gbase = pb + (size_t)(Lr + l - 1) * plane;      // G^{l-1}
        // ---- base G^{l-1} rows of the nodes at distance l+1 -> buffer (issued first)
        uint4 cvv[kIncCopy];
        int cdst[kIncCopy];
        int ctot = 0;
        {
          int cst[SM + 1];
          cst[0] = 0;
#pragma unroll
          for (int w = 0; w < SM; ++w)
            cst[w + 1] = cst[w] + (w < nsw ? (s_cnt[w][l + 1] - s_cnt[w][l]) * VPR : 0);
          ctot = cst[SM];
          // copy item idx -> (source vector, byte offset of the destination in LDS)
          auto locate = [&](int idx, const uint4*& src) {
            int w = 0, start = 0;
#pragma unroll
            for (int u = 1; u < SM; ++u)
              if (idx >= cst[u]) { w = u; start = cst[u]; }
            const int rel = idx - start;
            const int rr = s_cnt[w][l] + rel / VPR, v = rel % VPR;
            const int nd = tab[w * ig.tabw + rr];
            src = reinterpret_cast<const uint4*>(Gbase + (size_t)nd * F) + v;
            return ig.off_buf + ((w * ig.rows + rr) * ig.row_elems) * (int)sizeof(Acc) + 16 * v;
          };
#pragma unroll
          for (int u = 0; u < kIncCopy; ++u) {
            const int idx = threadIdx.x + u * bd;
            const uint4* src = reinterpret_cast<const uint4*>(Gbase);   // in-bounds placeholder
            cdst[u] = -1;
            if (idx < ctot) cdst[u] = locate(idx, src);
            cvv[u] = *src;   // unconditional, so the value stays in registers
          }
          for (int idx = threadIdx.x + kIncCopy * bd; idx < ctot; idx += bd) {   // rare: large rings
            const uint4* src;
            const int o = locate(idx, src);
            *reinterpret_cast<uint4*>(smem + o) = *src;
          }
        }
        // ---- this wave's tiles: inputs
        Acc h[MAXT][NS];
        int trow[MAXT], tsw[MAXT];
        bool tok[MAXT];
#pragma unroll
        for (int k = 0; k < MAXT; ++k) {
          const int g = wv + k * nw;
          const int w = g % nsw, tt = g / nsw;
          tsw[k] = w;
          tok[k] = tt * 16 < s_cnt[w][l];
          trow[k] = tt * 16 + col;
        }
        auto load_h = [&](int k) {
          const int w = tsw[k], r = trow[k];
          const int cl = s_cnt[w][l], cp = s_cnt[w][l - 1];
          const int nd = r < cl ? tab[w * ig.tabw + r] : -1;
          if (l == 1) {
            const int x = nd >= 0 ? xnew(w, nd) : 0;
#pragma unroll
            for (int i = 0; i < NS; ++i) h[k][i] = nd >= 0 ? semb[x * F + P::lc(q, i)] : (Acc)0;
          } else if (r < cp) {
            lds_read<Acc, NS>(buf + ((size_t)w * ig.rows + r) * ig.row_elems + q * NS, h[k]);   // H'^{l-1}
          } else if (nd >= 0) {
            gmem_read<Acc, NS>(Hbase + (size_t)nd * F + q * NS, h[k]);                       // base H^{l-1}
          } else {
#pragma unroll
            for (int i = 0; i < NS; ++i) h[k][i] = (Acc)0;
          }
        };
        // ---- products: self -> registers, message -> buffer rows [0, |C_l|) in place
        CF acc[MAXT][MT];
#pragma unroll
        for (int k = 0; k < MAXT; ++k) {
          if (!tok[k]) continue;
          load_h(k);
          const int w = tsw[k], r = trow[k];
          const bool wr = r < s_cnt[w][l];
          Acc* row = buf + ((size_t)w * ig.rows + r) * ig.row_elems + q * NS;
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            CF a, gs = CF{0, 0, 0, 0};
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) a[rr] = bias[4 * t + rr];
#pragma unroll
            for (int st = 0; st < KSB; ++st) {
              const auto bop = P::make_b(&h[k][st * VEC]);
              gs = P::mma(P::load_a(afrag(0, st, t)), bop, gs);
              a = P::mma(P::load_a(afrag(1, st, t)), bop, a);
            }
            acc[k][t] = a;
            if (wr) {
              Acc gm[4] = {gs[0], gs[1], gs[2], gs[3]};
              lds_write<Acc, 4>(row + 4 * t, gm);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kIncCopy; ++u)
          if (cdst[u] >= 0) *reinterpret_cast<uint4*>(smem + cdst[u]) = cvv[u];
        __syncthreads();   // every G^{l-1} row of every swap is in its buffer
        // ---- gather, activation; readout difference at the last layer
        if (l == Lr && lane == 0)
          for (int w = 0; w < nsw; ++w) red[(2 * w) * kMaxWaves + wv] = red[(2 * w + 1) * kMaxWaves + wv] = 0.0;
        Acc hn[MAXT][NS];
#pragma unroll
        for (int k = 0; k < MAXT; ++k) {
          if (!tok[k]) continue;
          const int w = tsw[k], r = trow[k];
          const int cl = s_cnt[w][l];
          const int* tw = tab + w * ig.tabw;
          const int nd = r < cl ? tw[r] : -1;
          const Acc* bw = buf + (size_t)w * ig.rows * ig.row_elems;
          Acc hb[NS];
          if (l == Lr && nd >= 0) gmem_read<Acc, NS>(pb + (size_t)(Lr - 1) * plane + (size_t)nd * F + q * NS, hb);
          Acc m[NS];
#pragma unroll
          for (int i = 0; i < NS; ++i) m[i] = (Acc)0;
          if (nd >= 0) {
            const int* nbp = tw + inc.r4 + r * dm;
            for (int d = 0; d < dm; d += 4) {
              const int4 pv = *reinterpret_cast<const int4*>(nbp + d);
              const int pc[4] = {pv.x, pv.y, pv.z, pv.w};
              const Acc* wp = sev + nd * dm + d;
              const Acc wt[4] = {wp[0], wp[1], wp[2], wp[3]};
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                Acc rowv[NS];
                lds_read<Acc, NS>(bw + pc[u] * ig.row_elems + q * NS, rowv);
#pragma unroll
                for (int i = 0; i < NS; ++i) m[i] += wt[u] * rowv[i];
              }
            }
          }
#pragma unroll
          for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) hn[k][4 * t + rr] = P::act(acc[k][t][rr] + m[4 * t + rr]);
          if (l == Lr) {
            double pa = 0.0, pp = 0.0;
            if (nd >= 0) {
              // readout difference of this node, each side formed as in the full evaluation
              Acc ta1 = 0, tp1 = 0, ta0 = 0, tp0 = 0;
#pragma unroll
              for (int i = 0; i < NS; ++i) {
                const int f = P::lc(q, i);
                ta1 += (Acc)shead[f] * hn[k][i];
                tp1 += (Acc)shead[F + 3 + f] * hn[k][i];
                ta0 += (Acc)shead[f] * hb[i];
                tp0 += (Acc)shead[F + 3 + f] * hb[i];
              }
              pa = (double)ta1 - (double)ta0;
              pp = (double)tp1 - (double)tp0;
            }
            pa = wave_sum(pa);
            pp = wave_sum(pp);
            if (lane == 0) {
              red[(2 * w) * kMaxWaves + wv] += pa;
              red[(2 * w + 1) * kMaxWaves + wv] += pp;
            }
          }
        }
        if (l < Lr) {
          __syncthreads();   // every gather read of the buffers is done
#pragma unroll
          for (int k = 0; k < MAXT; ++k) {
            if (!tok[k]) continue;
            const int w = tsw[k], r = trow[k];
            if (r < s_cnt[w][l]) lds_write<Acc, NS>(buf + ((size_t)w * ig.rows + r) * ig.row_elems + q * NS, hn[k]);
          }
        }
      }
      __syncthreads();   // readout partials of every wave
      if ((int)threadIdx.x < nsw) {
        const int w = threadIdx.x;
        double da = 0.0, dp = 0.0;
        for (int v = 0; v < nw; ++v) {
          da += red[(2 * w) * kMaxWaves + v];
          dp += red[(2 * w + 1) * kMaxWaves + v];
        }
        const double mm = exp(da);
        double sn, cs;
        sincos(dp, &sn, &cs);
        const double xr = mm * cs, xi = mm * sn;
        double t = sr + xr;
        cr += (fabs(sr) >= fabs(xr)) ? ((sr - t) + xr) : ((xr - t) + sr);
        sr = t;
        t = si + xi;
        ci += (fabs(si) >= fabs(xi)) ? ((si - t) + xi) : ((xi - t) + si);
        si = t;
      }
    }
    // combine the slots in slot order
    if ((int)threadIdx.x < SM) {
      s_acc[threadIdx.x][0] = sr; s_acc[threadIdx.x][1] = cr;
      s_acc[threadIdx.x][2] = si; s_acc[threadIdx.x][3] = ci;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double tr = 0, tcr = 0, ti = 0, tci = 0;
      for (int w = 0; w < min(S, SM); ++w) {
        double x = s_acc[w][0];
        double t = tr + x;
        tcr += (fabs(tr) >= fabs(x)) ? ((tr - t) + x) : ((x - t) + tr);
        tr = t;
        tcr += s_acc[w][1];
        x = s_acc[w][2];
        t = ti + x;
        tci += (fabs(ti) >= fabs(x)) ? ((ti - t) + x) : ((x - t) + ti);
        ti = t;
        tci += s_acc[w][3];
      }
      double* o = partial + 4 * (size_t)it;
      o[0] = tr; o[1] = tcr; o[2] = ti; o[3] = tci;
      cnt[it] = nanti;
    }
    __syncthreads();
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
