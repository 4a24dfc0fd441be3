// Incremental local energy: log psi(s^ij) - log psi(s) from the swapped sites'
// receptive field only.
//
// Exchanging the spins of bond (i, j) changes the layer-l embedding of exactly
// the nodes within graph distance l of {i, j} (the ball C_l), because layer l of
// Eq. 1 reads a node and its neighbours.  With the base planes of sample s
// (layer outputs H^l and message products G^l = H^l W_msg, written by the base
// pass), layer l is recomputed for the rows of C_l only:
//   G'_m = H'^{l-1}_m W_msg                  for m in C_{l-1}
//   P'_n = b + H'^{l-1}_n W_self + sum_d A_hat[n][d] G'^{l-1}_{nbr}   for n in C_l
// where every input outside C_{l-1} is read from the base planes.  The rows are
// computed with the same instructions, operand order and reduction order as the
// full evaluation, so they are bit-identical to it, and
//   Delta = (v_a + i v_p) . sum_{n in C_L} (H'^L_n - H^L_n).
// The ball tables are built on the host per bond; row sets are padded to tiles
// of 16 with rows whose node id is -1.
#pragma once

#include "gna_kernels.h"

namespace gna {

struct IncNet {
  int n, F, L, dmax;
  int rows_max;              // largest padded ball, rows of the LDS buffers
  const int* ball_off;       // [ne][L+1] first row of layer l of bond e
  const int* ball_cnt;       // [ne][L+1] padded row count (multiple of 16)
  const int* ball_node;      // [rows] node id or -1
  const int* ball_self;      // [rows] layer l >= 1: row of the node in C_{l-1}, or -1-node
  const int* ball_nb;        // [rows][dmax] layer l >= 1: row in C_{l-1}, or -1-node (base)
  const int* ell_idx;        // [npad][dmax] (for the adjacency weights)
  const void* ell_val;       // [npad][dmax] Acc
};

// LDS layout of k_eloc_inc (byte offsets)
struct IncGeo {
  int nw;          // waves per workgroup
  int row_elems;   // LDS row stride in Acc elements
  int off_w, off_hc, off_gc, off_sp, off_red, off_bias, off_emb, off_head;
  int off_tab;     // one bond's ball tables (node, self, neighbour codes)
  int tab_ints;    // capacity in ints
  int xcd;         // items are grouped per XCD (blocks b with equal b % xcd share a sample)
  int lds_bytes;
};

template <class P, int F, int MAXT>
__global__ __launch_bounds__(512) void k_eloc_inc(Net net, IncNet inc, IncGeo ig, const int8_t* __restrict__ spins,
                                                  int B, const typename P::Acc* __restrict__ planes, int n_chunks,
                                                  int chunk, double* __restrict__ partial, int* __restrict__ cnt) {
  using Acc = typename P::Acc;
  using WT = typename P::WT;
  using AF = typename P::AF;
  using BF = typename P::BF;
  using CF = typename P::CF;
  constexpr int NS = F / 4, MT = F / 16, KSB = F / P::KS, VEC = P::VEC;
  extern __shared__ __align__(16) unsigned char smem[];
  WT* wl = reinterpret_cast<WT*>(smem + ig.off_w);
  Acc* Hc = reinterpret_cast<Acc*>(smem + ig.off_hc);   // H' rows of the previous layer's ball
  Acc* Gc = reinterpret_cast<Acc*>(smem + ig.off_gc);   // G' rows of the previous layer's ball
  int8_t* sp = reinterpret_cast<int8_t*>(smem + ig.off_sp);
  double* red = reinterpret_cast<double*>(smem + ig.off_red);
  Acc* sbias = reinterpret_cast<Acc*>(smem + ig.off_bias);
  Acc* semb = reinterpret_cast<Acc*>(smem + ig.off_emb);
  double* shead = reinterpret_cast<double*>(smem + ig.off_head);

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q = lane >> 4, col = lane & 15;
  const int nw = ig.nw, Lr = net.L;
  const size_t plane = (size_t)net.g.npad * F;
  const Acc* ev = reinterpret_cast<const Acc*>(inc.ell_val);

  // stage weights (tied: one layer) and the small tables
  {
    const int nwt = 2 * F * F;
    const WT* src = reinterpret_cast<const WT*>(net.wfrag);
    for (int k = threadIdx.x; k < nwt; k += blockDim.x) wl[k] = src[k];
    for (int k = threadIdx.x; k < F; k += blockDim.x)
      sbias[k] = reinterpret_cast<const Acc*>(net.bias)[P::lc(k / NS, k % NS)];   // slot order
    for (int k = threadIdx.x; k < 2 * F; k += blockDim.x) semb[k] = reinterpret_cast<const Acc*>(net.emb)[k];
    for (int k = threadIdx.x; k < F + 3; k += blockDim.x) {
      shead[k] = net.head_a[k];
      shead[F + 3 + k] = net.head_p[k];
    }
  }
  __syncthreads();
  auto afrag = [&](int blk, int st, int t) { return wl + (((blk * KSB + st) * MT + t) * 64 + lane) * VEC; };
  const Acc* bias = sbias + q * NS;

  int* tab = reinterpret_cast<int*>(smem + ig.off_tab);
  // XCD-aware order: the blocks of one XCD (equal blockIdx % xcd) walk the chunks of
  // the same samples together, so a sample's base planes stay in that XCD's L2
  const int X = ig.xcd;
  const int per_x = gridDim.x / X;
  const int xid = blockIdx.x % X, slot = blockIdx.x / X;
  const long long per_xcd_items = (long long)((B - xid + X - 1) / X) * n_chunks;
  for (long long j = slot; j < per_xcd_items; j += per_x) {
    const int b = xid + X * (int)(j / n_chunks), c = (int)(j % n_chunks);
    const int it = b * n_chunks + c;
    for (int k = threadIdx.x; k < net.n; k += blockDim.x) sp[k] = spins[(size_t)b * net.n + k];
    __syncthreads();
    const Acc* pb = planes + (size_t)b * 2 * Lr * plane;
    double sr = 0, cr = 0, si = 0, ci = 0;
    int ne = 0;
    const int e0 = c * chunk, e1 = min(net.ne, e0 + chunk);
    for (int e = e0; e < e1; ++e) {
      const int2 ij = net.edges[e];
      if (sp[ij.x] == sp[ij.y]) continue;   // uniform across the workgroup
      // this bond's tables -> LDS (rows of all layers: node, self code, neighbour codes)
      const int* gofs = inc.ball_off + e * (Lr + 1);
      const int* gcnt = inc.ball_cnt + e * (Lr + 1);
      const int row0 = gofs[0], nrows = gofs[Lr] + gcnt[Lr] - row0;
      const int dm = inc.dmax;
      for (int k = threadIdx.x; k < nrows; k += blockDim.x) {
        tab[k] = inc.ball_node[row0 + k];
        tab[nrows + k] = inc.ball_self[row0 + k];
      }
      for (int k = threadIdx.x; k < nrows * dm; k += blockDim.x) tab[2 * nrows + k] = inc.ball_nb[(size_t)row0 * dm + k];
      __syncthreads();
      int boff[17], bcnt[17];
#pragma unroll 1
      for (int l = 0; l <= Lr; ++l) {
        boff[l] = gofs[l] - row0;
        bcnt[l] = gcnt[l];
      }
      // spin of node nd in the exchanged configuration
      auto xnew = [&](int nd) {
        const int8_t v = (nd == ij.x) ? sp[ij.y] : ((nd == ij.y) ? sp[ij.x] : sp[nd]);
        return v > 0 ? 1 : 0;
      };
      double pa = 0.0, pp = 0.0;
      for (int l = 1; l <= Lr; ++l) {
        const int* rows_prev = tab + boff[l - 1];
        const int tprev = bcnt[l - 1] / 16;
        const int* rows_cur = tab + boff[l];
        const int* self_cur = tab + nrows + boff[l];
        const int* nb_cur = tab + 2 * nrows + (size_t)boff[l] * dm;
        const int tcur = bcnt[l] / 16;
        const Acc* Hbase = pb + (size_t)(l - 2) * plane;           // H^{l-1} (l >= 2)
        const Acc* Gbase = pb + (size_t)(Lr + l - 1) * plane;      // G^{l-1}
        // phase A: message product of the previous ball's rows -> Gc
        for (int tt = wv; tt < tprev; tt += nw) {
          const int r = tt * 16 + col;
          const int nd = rows_prev[r];
          Acc h[NS];
          if (l == 1) {
            const int x = nd >= 0 ? xnew(nd) : 0;
#pragma unroll
            for (int i = 0; i < NS; ++i) h[i] = nd >= 0 ? semb[x * F + P::lc(q, i)] : (Acc)0;
          } else {
            lds_read<Acc, NS>(Hc + r * ig.row_elems + q * NS, h);
          }
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            CF a = CF{0, 0, 0, 0};
#pragma unroll
            for (int st = 0; st < KSB; ++st) a = P::mma(P::load_a(afrag(0, st, t)), P::make_b(&h[st * VEC]), a);
            Acc gm[4] = {a[0], a[1], a[2], a[3]};
            lds_write<Acc, 4>(Gc + r * ig.row_elems + q * NS + 4 * t, gm);
          }
        }
        // phase B: self product of this ball's rows (registers)
        CF acc[MAXT][MT];
#pragma unroll
        for (int k = 0; k < MAXT; ++k) {
          const int tt = wv + k * nw;
          if (tt >= tcur) break;
          const int r = tt * 16 + col;
          const int nd = rows_cur[r];
          const int src = self_cur[r];
          Acc h[NS];
          if (l == 1) {
            const int x = nd >= 0 ? xnew(nd) : 0;                       // embedding, exchanged spins
#pragma unroll
            for (int i = 0; i < NS; ++i) h[i] = nd >= 0 ? semb[x * F + P::lc(q, i)] : (Acc)0;
          } else if (src >= 0) {
            lds_read<Acc, NS>(Hc + src * ig.row_elems + q * NS, h);   // changed at layer l-1
          } else {
            const int m = -1 - src;
            lds_read<Acc, NS>(Hbase + (size_t)m * F + q * NS, h);     // base plane
          }
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            CF a;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) a[rr] = bias[4 * t + rr];
#pragma unroll
            for (int st = 0; st < KSB; ++st) a = P::mma(P::load_a(afrag(1, st, t)), P::make_b(&h[st * VEC]), a);
            acc[k][t] = a;
          }
        }
        __syncthreads();   // Gc complete; Hc no longer read this layer
        // phase C: gather, activation; rows of C_l go to Hc
        Acc hnew[MAXT][NS];
#pragma unroll
        for (int k = 0; k < MAXT; ++k) {
          const int tt = wv + k * nw;
          if (tt >= tcur) break;
          const int r = tt * 16 + col;
          const int nd = rows_cur[r];
          Acc m[NS];
#pragma unroll
          for (int i = 0; i < NS; ++i) m[i] = (Acc)0;
          if (nd >= 0) {
            for (int d = 0; d < inc.dmax; ++d) {
              const int code = nb_cur[(size_t)r * inc.dmax + d];
              const Acc w = ev[nd * inc.dmax + d];
              Acc row[NS];
              if (code >= 0) lds_read<Acc, NS>(Gc + code * ig.row_elems + q * NS, row);
              else lds_read<Acc, NS>(Gbase + (size_t)(-1 - code) * F + q * NS, row);
#pragma unroll
              for (int i = 0; i < NS; ++i) m[i] += w * row[i];
            }
          }
#pragma unroll
          for (int t = 0; t < MT; ++t)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) hnew[k][4 * t + rr] = P::act(acc[k][t][rr] + m[4 * t + rr]);
          if (l == Lr && nd >= 0) {
            // readout difference of this node, each side formed as in the full evaluation
            Acc hb[NS];
            lds_read<Acc, NS>(pb + (size_t)(Lr - 1) * plane + (size_t)nd * F + q * NS, hb);
            Acc ta1 = 0, tp1 = 0, ta0 = 0, tp0 = 0;
#pragma unroll
            for (int i = 0; i < NS; ++i) {
              const int f = P::lc(q, i);
              ta1 += (Acc)shead[f] * hnew[k][i];
              tp1 += (Acc)shead[F + 3 + f] * hnew[k][i];
              ta0 += (Acc)shead[f] * hb[i];
              tp0 += (Acc)shead[F + 3 + f] * hb[i];
            }
            pa += (double)ta1 - (double)ta0;
            pp += (double)tp1 - (double)tp0;
          }
        }
        if (l < Lr) {
          __syncthreads();   // every read of Hc (phase B) and Gc (phase C) is done
#pragma unroll
          for (int k = 0; k < MAXT; ++k) {
            const int tt = wv + k * nw;
            if (tt >= tcur) break;
            lds_write<Acc, NS>(Hc + (tt * 16 + col) * ig.row_elems + q * NS, hnew[k]);
          }
          __syncthreads();
        }
      }
      pa = wave_sum(pa);
      pp = wave_sum(pp);
      if (lane == 0) {
        red[wv] = pa;
        red[kMaxWaves + wv] = pp;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double da = 0.0, dp = 0.0;
        for (int w = 0; w < nw; ++w) {
          da += red[w];
          dp += red[kMaxWaves + w];
        }
        const double mm = exp(da);
        double sn, cs;
        sincos(dp, &sn, &cs);
        // compensated sums, as in the full kernel
        const double xr = mm * cs, xi = mm * sn;
        double t = sr + xr;
        cr += (fabs(sr) >= fabs(xr)) ? ((sr - t) + xr) : ((xr - t) + sr);
        sr = t;
        t = si + xi;
        ci += (fabs(si) >= fabs(xi)) ? ((si - t) + xi) : ((xi - t) + si);
        si = t;
        ++ne;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double* o = partial + 4 * (size_t)it;
      o[0] = sr; o[1] = cr; o[2] = si; o[3] = ci;
      cnt[it] = ne;
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
