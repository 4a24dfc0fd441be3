// Layer-pipelined incremental evaluation (local energy and Metropolis sweeps).
//
// The ball evaluation of an exchange (Section 3's log psi(s^ij) - log psi(s) from
// the receptive field of the exchanged pair, as in gna_inc.h) has L dependent
// layers of 1 to a few 16-row tiles each.  Advancing one exchange at a time
// leaves most waves of a workgroup idle and pays two barriers per layer and
// exchange.  Here a workgroup keeps D = L + 1 + extra jobs in flight whose layers
// are staggered: job slot j is set up at ticks T = j mod D, its table is staged at
// tick T + extra and it computes layer l at tick T + extra + l.  A tick has two
// barriers, and between them every job in flight advances one layer, so a tick
// carries the tiles of all L layers (one job each) and a job costs two barriers
// instead of 2L.
//
// One wave (the setup wave) prepares the jobs; the others compute tiles from a
// schedule fixed by the host, (tick mod D, wave, register k) -> (job slot, tile).
// A tile belongs to the same wave and registers for the whole job, so a layer's
// output rows stay in registers (hn) as the next layer's input.
//   phase A  compute waves: message products G'^{l-1} = H'^{l-1} W_msg into the
//            job's LDS rows; this tick's ring rows stored into LDS (requested in
//            the last tick); base H^l rows of ring l+1 requested into the lanes of
//            hn that layer l+1 reads from them.  Setup wave: a new job's bond table
//            (requested in the last tick) stored.
//   barrier
//   phase B  compute waves: gather of A_hat G' over the job's LDS rows, self
//            product, activation, readout difference at layer L; the new table's
//            list positions turned into LDS rows; the next tick's ring rows
//            requested.  Setup wave: the readout difference of the job that
//            finished its layer L last tick (written out for the local energy, whose
//            terms k_eloc_terms sums in bond order; or the sampler's decision on
//            it), the slot's next job, the next table requested, the list of the
//            ring rows of the tick after next.
//   barrier
// The setup wave's work is on the critical path of a tick when the compute waves
// have few tiles each: it keeps the job state in registers (LDS round trips are
// long under the compute waves' traffic) and the tag conversion, which needs none
// of that state, is spread over the compute waves with fewer tiles in the phase.
// LDS rows of a job are not one buffer sized for the largest ball: rows of list
// positions [0, |C_2|) (computed at layer 1 from the spins) and of each ring
// [|C_{s-1}|, |C_s|), s >= 3 (copied from the base planes for the gather of
// layer s-1) live in pools.  Pool pi holds positions of ring pi + 2 (pi = 0: the
// prefix [0, |C_2|)) from layer pi + 1 to layer L, i.e. during L - pi ticks; since
// jobs start one tick apart, L - pi slots of the pool suffice, slot = tick mod
// (L - pi).  A bond's table carries each position's pool and offset, which the
// compute waves turn into LDS rows when the job's table is staged.
//
// In the sampler a proposal writes its recomputed rows into the chain's planes as
// they are produced (rows read later in the same evaluation are never among them),
// and a rejected proposal is followed by a restore job, the same ball for the
// chain's configuration, which rewrites the old rows bit for bit.  At the
// benchmark's near-uniform amplitudes almost every anti-aligned proposal is
// accepted, so restores are rare (writing only after an accept would double the
// jobs there).
//
// Arithmetic is the same instruction sequence per row as the full evaluation and
// the group kernel (the rows are bit-identical); only the order of the FP64
// readout sums over tiles and waves differs.
#pragma once

#include "gna_inc.h"

namespace gna {

constexpr int kPipeMaxD = 16;        // job slots
constexpr int kPipeMaxK = 8;         // tile registers per wave
constexpr int kPipeMaxL = 14;        // layers (the table header holds |C_0| .. |C_{L+1}|)
constexpr int kPipeHdr = 16;         // uint16 header entries of a bond table
constexpr int kPipeTabVec = 4;       // 16-byte table vectors per lane of the setup wave
constexpr int kPipeMaskWords = 64;   // anti-aligned bond mask of a work item (2048 bonds, a word per lane)

struct PipeGeo {
  int nw, D, extra, sw;     // waves, job slots, idle ticks between setup and layer 1, setup wave
  int row_elems;            // LDS row stride (Acc elements)
  int pool_base[kPipeMaxL], pool_cnt[kPipeMaxL], pool_rows[kPipeMaxL];
  int tabw;                 // uint16 entries of a bond table (global and LDS; multiple of 8)
  int r8;                   // list positions per bond (multiple of 8)
  int ntab;                 // LDS tables (L + 1)
  int spw;                  // bytes per spin row in LDS
  int off_w, off_arena, off_tab, off_sp, off_red, off_bias, off_emb, off_head, off_ev, off_edges;
  int off_rows;             // ring rows of a tick's copies: [2 (tick parity)][rows_max] uint2
  int rows_max;             // ring rows copied in one tick at most
  int xcd;
  int lds_bytes;
};

// job state of a workgroup (LDS)
struct PipeState {
  // per job slot, written by the setup wave (which keeps its own copies in registers)
  // and read by the compute waves
  int valid[kPipeMaxD];
  int flags[kPipeMaxD];
  int2 ij[kPipeMaxD];
  long long pboff[kPipeMaxD];
  int t1[kPipeMaxD];                          // table tick of the job
  int tbo[kPipeMaxD];                         // its LDS table (uint16 offset), from the table tick on
  unsigned short hdr[kPipeMaxD][kPipeHdr];    // |C_0| .. |C_{L+1}| of its bond, from the table tick on
  int rowbase[kPipeMaxL];                     // first arena row of each pool slot of the job staged
  unsigned short rb[kPipeMaxD][kPipeMaxL];    // setup wave: the same for each job slot's job
  int conv;                                   // LDS table staged this tick (uint16 offset), or -1
  int nrows[2];                               // ring rows copied in a tick (by tick parity)
  int done;
};

// ReLU and layer normalisation of a node row in place: the same operations, in the
// same order, as relu_ln_row (its y and h in the one array)
template <class Acc, int NS>
__device__ __forceinline__ void relu_ln_inplace(Acc (&x)[NS]) {
  constexpr int F = 4 * NS;
  Acc s = 0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    x[i] = x[i] > (Acc)0 ? x[i] : (Acc)0;
    s += x[i];
  }
  const Acc mu = quad_sum(s) / (Acc)F;
  Acc v = 0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const Acc d = x[i] - mu;
    v += d * d;
  }
  const Acc r = (Acc)1 / sqrt(quad_sum(v) / (Acc)F + (Acc)kLnEps);
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = (x[i] - mu) * r;
}

// A tile's layer input is held in registers as its MFMA B operands: make_b of the
// row's NS values, K step by K step, in the first KSB * sizeof(BF) bytes of the NS
// words (the rest unused). Built once where the input is produced instead of before
// each of the two products that read it.
template <class P, int NS>
__device__ __forceinline__ void pipe_to_ops(const typename P::Acc (&x)[NS], typename P::Acc (&h)[NS]) {
  using BF = decltype(P::make_b((const typename P::Acc*)nullptr));
  constexpr int KSB = NS / P::VEC;
  static_assert(sizeof(typename P::Acc) == 4 && sizeof(BF) * KSB <= 4 * NS, "operands fit the input's words");
  BF b[KSB];
#pragma unroll
  for (int stp = 0; stp < KSB; ++stp) b[stp] = P::make_b(&x[stp * P::VEC]);
  __builtin_memcpy(h, b, sizeof(BF) * KSB);
}

template <class P, int F, int MAXT, int NT, int NCOPY, bool SWEEP>
__device__ __forceinline__ void pipe_body(const Net& net, const IncNet& inc, const PipeGeo& pg,
                                          const uint2* __restrict__ sched, const uint16_t* __restrict__ gtab,
                                          int8_t* spins, int B, typename P::Acc* planes, int n_chunks, int chunk,
                                          double* __restrict__ terms, int n_sweeps,
                                          unsigned long long seed, unsigned long long counter_base,
                                          const unsigned long long* __restrict__ counter_dev,
                                          int* __restrict__ n_accept) {
  using Acc = typename P::Acc;
  using CF = typename P::CF;
  using WT = typename P::WT;
  using V4 = unsigned int __attribute__((ext_vector_type(4)));
  constexpr int NS = F / 4, MT = F / 16, KSB = F / P::KS, VEC = P::VEC;
  constexpr int VPR = F * (int)sizeof(Acc) / 16;   // 16-byte vectors per row
  static_assert(sizeof(Acc) == 4, "FP32 activations (FP64 is not pipelined)");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ PipeState st;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q = lane >> 4, col = lane & 15;
  const int nw = pg.nw, D = pg.D, extra = pg.extra, Lr = net.L, dm = inc.dmax, r8 = pg.r8;
  const int ntab = pg.ntab, tabw = pg.tabw;
  const size_t plane = (size_t)net.g.npad * F;
  const long long per = 2LL * Lr * (long long)plane;   // planes of one sample / chain
  const int row_bytes = pg.row_elems * (int)sizeof(Acc);

  WT* wl = reinterpret_cast<WT*>(smem + pg.off_w);
  Acc* arena = reinterpret_cast<Acc*>(smem + pg.off_arena);
  uint16_t* tabs = reinterpret_cast<uint16_t*>(smem + pg.off_tab);
  int8_t* sp = reinterpret_cast<int8_t*>(smem + pg.off_sp);
  double* red = reinterpret_cast<double*>(smem + pg.off_red);   // [tick parity][2][kMaxWaves]
  Acc* sbias = reinterpret_cast<Acc*>(smem + pg.off_bias);
  Acc* semb = reinterpret_cast<Acc*>(smem + pg.off_emb);
  double* shead = reinterpret_cast<double*>(smem + pg.off_head);
  Acc* sev = reinterpret_cast<Acc*>(smem + pg.off_ev);
  unsigned* sedge = reinterpret_cast<unsigned*>(smem + pg.off_edges);   // i | j << 16

  // ---- weights, node tables and bond endpoints -> LDS
  {
    const WT* src = reinterpret_cast<const WT*>(net.wfrag);
    for (int k = threadIdx.x; k < P::WBLK * 2 * F * F; k += NT) wl[k] = src[k];
    for (int k = threadIdx.x; k < F; k += NT) sbias[k] = reinterpret_cast<const Acc*>(net.bias)[P::lc(k / NS, k % NS)];
    // the embedding of spin value s as lane group q's B operands, at semb + (2q + s) NS
    for (int k = threadIdx.x; k < 8; k += NT) {
      const int s = k & 1, qq = k >> 1;
      Acc x[NS], h[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        x[i] = reinterpret_cast<const Acc*>(net.emb)[s * F + P::lc(qq, i)];
        h[i] = (Acc)0;
      }
      pipe_to_ops<P, NS>(x, h);
#pragma unroll
      for (int i = 0; i < NS; ++i) semb[k * NS + i] = h[i];
    }
    for (int k = threadIdx.x; k < F; k += NT) {
      const int f = P::lc(k / NS, k % NS);
      shead[k] = net.head_a[f];
      shead[F + k] = net.head_p[f];
    }
    const Acc* ev = reinterpret_cast<const Acc*>(inc.ell_val);
    for (int k = threadIdx.x; k < net.n * dm; k += NT) sev[k] = ev[k];
    for (int k = threadIdx.x; k < net.ne; k += NT) {
      const int2 ij = net.edges[k];
      sedge[k] = (unsigned)ij.x | ((unsigned)ij.y << 16);
    }
    for (int k = threadIdx.x; k < 4 * kMaxWaves; k += NT) red[k] = 0.0;
  }
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const long long total = (long long)n_sweeps * net.n;
  if constexpr (SWEEP) {
    if (counter_dev) counter_base += *counter_dev;   // graph replays read the current base
  }
  // local energy: XCD-aware order of the work items (as the group kernel)
  const int X = pg.xcd;
  const int per_x = gridDim.x / X;
  const int xid = blockIdx.x % X, slotx = blockIdx.x / X;
  const long long per_xcd_items = SWEEP ? 0 : (long long)((B - xid + X - 1) / X) * n_chunks;
  if (threadIdx.x < kPipeMaxD) st.valid[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    st.done = 0;
    st.nrows[0] = st.nrows[1] = 0;
  }
  if constexpr (SWEEP) {   // the slots' first chains: chain blockIdx.x + j gridDim.x in slot j
    for (int j = 0; j < D; ++j) {
      const int b = blockIdx.x + j * gridDim.x;
      if (b < B)
        for (int k = threadIdx.x; k < net.n; k += NT) sp[j * pg.spw + k] = spins[(size_t)b * net.n + k];
    }
  }
  __syncthreads();

  // ---- ring-row copies (all waves share them): the rows of a tick are listed by the
  // setup wave (source 16-byte vector in the planes, destination byte offset in LDS);
  // item idx is vector idx % VPR of listed row idx / VPR
  const uint2* rows_l = reinterpret_cast<const uint2*>(smem + pg.off_rows);
  auto copy_find = [&](int pb, int nr, int idx, const V4*& src, int& dst) -> bool {
    const int rw = idx / VPR, v = idx % VPR;
    if (rw >= nr) return false;
    const uint2 rc = rows_l[pb * pg.rows_max + rw];
    src = reinterpret_cast<const V4*>(planes) + (size_t)rc.x + v;
    dst = (int)rc.y + 16 * v;
    return true;
  };
  V4 cvv[NCOPY];   // ring rows of the next tick, requested before the barrier
  int cdst[NCOPY];
#pragma unroll
  for (int u = 0; u < NCOPY; ++u) cdst[u] = -1;
  auto copy_store = [&](int T) {   // phase A: this tick's ring rows -> LDS
#pragma unroll
    for (int u = 0; u < NCOPY; ++u)
      if (cdst[u] >= 0) *reinterpret_cast<V4*>(smem + cdst[u]) = cvv[u];
    const int nr = __builtin_amdgcn_readfirstlane(st.nrows[T & 1]);
    for (int idx = threadIdx.x + NCOPY * NT; idx < nr * VPR; idx += NT) {   // rare: more rows than registers
      const V4* src;
      int dst;
      if (copy_find(T & 1, nr, idx, src, dst)) *reinterpret_cast<V4*>(smem + dst) = *src;
    }
  };
  // phase B: the next tick's ring rows -> registers; every thread issues NCOPY loads
  // (an idle one reads the first plane vector), so that waits for older loads can
  // leave these in flight
  auto copy_load = [&](int T) {
    const int nr = __builtin_amdgcn_readfirstlane(st.nrows[(T + 1) & 1]);
#pragma unroll
    for (int u = 0; u < NCOPY; ++u) {
      const V4* src = reinterpret_cast<const V4*>(planes);
      int dst = -1;
      if (!copy_find((T + 1) & 1, nr, threadIdx.x + u * NT, src, dst)) {
        src = reinterpret_cast<const V4*>(planes);
        dst = -1;
      }
      cvv[u] = *src;
      cdst[u] = dst;
    }
  };

  // phase B: the pool tags (pool << 12 | offset) of the table staged this tick turned
  // into LDS rows (the table is first read at the next tick), by the waves with fewer
  // tiles in this phase than the busiest (the schedule names them: nlight waves,
  // this wave's rank among them, 0xff when not one of them)
  auto tab_convert = [&](int nlight, int rank) {
    const int tbo = __builtin_amdgcn_readfirstlane(st.conv);
    if (tbo < 0 || rank == 0xff) return;
    uint16_t* tb = tabs + tbo;
    const int nv = tabw / 8;
    for (int v = (kPipeHdr + r8) / 8 + lane * nlight + rank; v < nv; v += 64 * nlight) {
      const V4 x = *reinterpret_cast<const V4*>(tb + 8 * v);
      unsigned o[4];
#pragma unroll
      for (int w4 = 0; w4 < 4; ++w4) {
        const unsigned lo = x[w4] & 0xffffu, hi = x[w4] >> 16;
        o[w4] = (unsigned)(st.rowbase[lo >> 12] + (int)(lo & 0xfffu)) |
                ((unsigned)(st.rowbase[hi >> 12] + (int)(hi & 0xfffu)) << 16);
      }
      *reinterpret_cast<V4*>(tb + 8 * v) = V4{o[0], o[1], o[2], o[3]};
    }
  };

  if (wv == pg.sw) {
    // ======================= the setup wave =======================
    // This wave's work is on the critical path of a tick, and it shares its SIMD
    // with compute waves: it issues at a higher priority than theirs.  The state of
    // job slot j sits in lane j of the registers below; the copies in LDS are for
    // the compute waves.  This wave writes LDS state and never waits for its own.
    __builtin_amdgcn_s_setprio(3);
    auto rl32 = [](int v, int j) { return __builtin_amdgcn_readlane(v, j); };
    auto rl64 = [](unsigned long long v, int j) {
      return (unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, j) |
             ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), j) << 32);
    };
    int r_valid = 0, r_t1 = 0, r_e = 0, r_tbo = 0, r_flags = 0, r_spb = -1, r_si = 0, r_sk = 0;
    unsigned r_ij = 0;
    unsigned long long r_pboff = 0;
    // sampler: the slot's chain, its accepted count, pending restore, next draw and
    // the uniform draw of the job in flight
    int r_chain = -1, r_nacc = 0, r_pend = -1;
    unsigned long long r_tstep = 0, r_u = 0;   // r_u: the double's bits
    if constexpr (SWEEP) {
      const int b = blockIdx.x + lane * gridDim.x;
      r_chain = (lane < D && b < B) ? b : -1;
    }
    // pool pi (lane pi): first LDS row and rows of a slot, slots, the slot of this tick
    int p_base = 0, p_rows = 0, p_cnt = 1, p_slot = 0;
#pragma unroll
    for (int i = 0; i < kPipeMaxL; ++i)
      if (lane == i && i < Lr) {
        p_base = pg.pool_base[i];
        p_rows = pg.pool_rows[i];
        p_cnt = pg.pool_cnt[i];
      }
    V4 tv[kPipeTabVec];   // a job's table (global -> registers), stored at its table tick
#pragma unroll
    for (int u = 0; u < kPipeTabVec; ++u) tv[u] = V4{0u, 0u, 0u, 0u};
    int tjob = -1;        // slot of the job whose table tv holds
    // local energy: the stream of work items of this workgroup; the current item's
    // anti-aligned bonds (bit per bond, word w in lane w) and, for items of at most
    // 64 bonds, each bond's endpoints (bond k in lane k)
    long long jj = (long long)slotx - per_x;
    int sb = -1, e0 = 0, clen = 0, cursor = 0;
    unsigned r_mask = 0u, r_bij = 0u;
    bool sdone = SWEEP;
    int inflight = 0;
    int8_t* ss = sp + D * pg.spw;   // the stream's sample
    for (int T = 0;; ++T) {
      const int tau = T % D;
      // ---- phase A: the table of the job whose table tick this is, stored as read (the
      // compute waves turn its pool tags into LDS rows in phase B), with the first LDS
      // row of each pool slot of the job
      if (tjob >= 0) {
        if (lane < Lr) {
          const int rbase = p_base + p_slot * p_rows;
          st.rowbase[lane] = rbase;
          st.rb[tjob][lane] = (unsigned short)rbase;
        }
        const int tbo = (T % ntab) * tabw;
        uint16_t* tb = tabs + tbo;
        const int nv = tabw / 8;
#pragma unroll
        for (int u = 0; u < kPipeTabVec; ++u) {
          const int v = lane + 64 * u;
          if (v < nv) *reinterpret_cast<V4*>(tb + 8 * v) = tv[u];
        }
        // the header (entries 0..15: table vectors 0 and 1, in lanes 0 and 1)
        if (lane < 2) {
          unsigned* hw = reinterpret_cast<unsigned*>(&st.hdr[tjob][8 * lane]);
#pragma unroll
          for (int w = 0; w < 4; ++w) hw[w] = tv[0][w];
        }
        if (lane == tjob) r_tbo = tbo;
        if (lane == 0) {
          st.tbo[tjob] = tbo;
          st.conv = tbo;
        }
      } else if (lane == 0) {
        st.conv = -1;
      }
      copy_store(T);
      p_slot = p_slot + 1 == p_cnt ? 0 : p_slot + 1;   // the pool slots of the next tick
      __syncthreads();
      // ---- phase B: this wave's readout slots, the job that left slot T mod D and
      // the slot's next job, the table of the job whose table tick is the next tick,
      // the next tick's ring rows
      if (lane == 0) {
        red[(T & 1) * 2 * kMaxWaves + wv] = 0.0;
        red[(T & 1) * 2 * kMaxWaves + kMaxWaves + wv] = 0.0;
      }
      const int j0 = tau;
      bool done = false;
      if (rl32(r_valid, j0)) {   // its layer L ran last tick
        // readout difference: the waves' partials, summed in a fixed order
        const double* rd = red + ((T - 1) & 1) * 2 * kMaxWaves;
        const double da = wave_sum_dpp(lane < nw ? rd[lane] : 0.0);
        const double dp = wave_sum_dpp(lane < nw ? rd[kMaxWaves + lane] : 0.0);
        if constexpr (SWEEP) {
          const int fl = rl32(r_flags, j0);
          if (fl & kJobReadout) {
            const double u = __longlong_as_double((long long)rl64(r_u, j0));
            if (u < exp(2.0 * da)) {   // accept: the planes already hold the new rows
              // the exchange (the pair's spins were read when the bond was drawn)
              const unsigned ij = (unsigned)rl32((int)r_ij, j0);
              const int si = rl32(r_si, j0), sk = rl32(r_sk, j0);
              if (lane == 0) {
                int8_t* sj = sp + j0 * pg.spw;
                sj[ij & 0xffffu] = (int8_t)sk;
                sj[ij >> 16] = (int8_t)si;
              }
              if (lane == j0) ++r_nacc;
            } else if (lane == j0) {
              r_pend = r_e;   // reject: the restore job of this bond comes next
            }
            if (lane == j0) ++r_tstep;
          } else if (lane == j0) {
            r_pend = -1;   // restored
          }
        } else if (lane == 0) {   // the exchange's term, summed in bond order by k_eloc_terms
          double* o = terms + 2 * ((size_t)rl32(r_spb, j0) * net.ne + rl32(r_e, j0));
          o[0] = da;
          o[1] = dp;
        }
        if (lane == 0) st.valid[j0] = 0;
        if (lane == j0) r_valid = 0;
        --inflight;
      }
      // ---- the next job of slot j0
      int e = -1;
      if constexpr (SWEEP) {
        int flags = 0;
        unsigned ij = 0u;
        while (rl32(r_chain, j0) >= 0) {
          const int b = rl32(r_chain, j0);
          const int pend = rl32(r_pend, j0);
          if (pend >= 0) {   // restore job: the chain's configuration, rows rewritten
            e = pend;
            ij = (unsigned)rl32((int)r_ij, j0);
            flags = 0;
            break;
          }
          // draws t, t+1, ... of the chain, 64 at a time; identity steps are skipped
          unsigned long long t = rl64(r_tstep, j0);
          const int8_t* sj = sp + j0 * pg.spw;
          while (t < (unsigned long long)total) {
            const unsigned long long tu = t + lane;
            const unsigned long long step = counter_base + tu;
            uint32_t c[4] = {(uint32_t)step, (uint32_t)(step >> 32), (uint32_t)b, 0u};
            philox4x32_10(c, k0, k1);
            const int eu = (int)(((unsigned long long)c[0] * (unsigned long long)net.ne) >> 32);
            const unsigned iju = sedge[eu];
            const int si = sj[iju & 0xffffu], sk = sj[iju >> 16];
            const bool anti = tu < (unsigned long long)total && si != sk;
            const unsigned long long m = __ballot(anti);
            if (m) {
              const int us = __builtin_ctzll(m);
              e = rl32(eu, us);
              ij = (unsigned)rl32((int)iju, us);
              const int siu = rl32(si, us), sku = rl32(sk, us);
              const uint32_t c1 = (uint32_t)rl32((int)c[1], us);
              t += us;
              const double u = ((double)c1 + 0.5) * 2.3283064365386963e-10;   // 2^-32
              if (lane == j0) {
                r_tstep = t;
                r_u = (unsigned long long)__double_as_longlong(u);
                r_si = siu;
                r_sk = sku;
              }
              break;
            }
            t += 64;
          }
          if (e >= 0) {
            flags = kJobSwap | kJobReadout;
            break;
          }
          // the chain is done: spins and acceptance count out, the slot's next chain in
          for (int k = lane; k < net.n; k += 64) spins[(size_t)b * net.n + k] = sj[k];
          const int nb = b + D * gridDim.x;
          const int nacc = rl32(r_nacc, j0);
          if (lane == 0 && n_accept) n_accept[b] = nacc;
          if (lane == j0) {
            r_chain = nb < B ? nb : -1;
            r_nacc = 0;
            r_pend = -1;
            r_tstep = 0;
          }
          if (nb < B)
            for (int k = lane; k < net.n; k += 64) sp[j0 * pg.spw + k] = spins[(size_t)nb * net.n + k];
          __builtin_amdgcn_s_waitcnt(0);
        }
        if (e >= 0) {
          const unsigned long long pbo = (unsigned long long)rl32(r_chain, j0) * (unsigned long long)per;
          if (lane == 0) {
            st.valid[j0] = 1;
            st.flags[j0] = flags;
            st.ij[j0] = make_int2((int)(ij & 0xffffu), (int)(ij >> 16));
            st.pboff[j0] = (long long)pbo;
            st.t1[j0] = T + extra;
          }
          if (lane == j0) {
            r_valid = 1;
            r_flags = flags;
            r_e = e;
            r_ij = ij;
            r_pboff = pbo;
            r_t1 = T + extra;
          }
          ++inflight;
        }
        if (inflight == 0) done = !__ballot(lane < D && r_chain >= 0);
      } else {
        int fidx = 0;
        while (!sdone) {
          // next anti-aligned bond of the current item at or after the cursor
          const int cw = cursor >> 5;
          unsigned mw = (lane >= cw && lane < ((clen + 31) >> 5)) ? r_mask : 0u;
          if (lane == cw) mw &= ~0u << (cursor & 31);
          const unsigned long long bal = __ballot(mw != 0u);
          if (bal) {
            const int fw = __builtin_ctzll(bal);
            fidx = fw * 32 + __builtin_ctz((unsigned)rl32((int)mw, fw));
            e = e0 + fidx;
            cursor = fidx + 1;
            break;
          }
          jj += per_x;
          if (jj >= per_xcd_items) {
            sdone = true;
            break;
          }
          const int b = xid + X * (int)(jj / n_chunks), cc = (int)(jj % n_chunks);
          e0 = cc * chunk;
          clen = max(0, min(net.ne, e0 + chunk) - e0);
          if (b != sb) {
            for (int k = lane; k < net.n; k += 64) ss[k] = spins[(size_t)b * net.n + k];
            __builtin_amdgcn_s_waitcnt(0);
            sb = b;
          }
          r_mask = 0u;
          for (int g = 0; g < clen; g += 64) {
            bool anti = false;
            unsigned ij = 0u;
            if (g + lane < clen) {
              ij = sedge[e0 + g + lane];
              anti = ss[ij & 0xffffu] != ss[ij >> 16];
            }
            if (g == 0) r_bij = ij;
            const unsigned long long m = __ballot(anti);
            if (lane == (g >> 5)) r_mask = (unsigned)m;
            if (lane == (g >> 5) + 1) r_mask = (unsigned)(m >> 32);
          }
          cursor = 0;
        }
        if (e >= 0) {
          if (rl32(r_spb, j0) != sb) {   // the slot's spin row
            const int* srcw = reinterpret_cast<const int*>(ss);
            int* dstw = reinterpret_cast<int*>(sp + j0 * pg.spw);
            for (int k = lane; k < pg.spw / 4; k += 64) dstw[k] = srcw[k];
          }
          const unsigned ij = clen <= 64 ? (unsigned)rl32((int)r_bij, fidx) : sedge[e];
          const unsigned long long pbo = (unsigned long long)sb * (unsigned long long)per;
          if (lane == 0) {
            st.valid[j0] = 1;
            st.flags[j0] = kJobSwap | kJobReadout;
            st.ij[j0] = make_int2((int)(ij & 0xffffu), (int)(ij >> 16));
            st.pboff[j0] = (long long)pbo;
            st.t1[j0] = T + extra;
          }
          if (lane == j0) {
            r_valid = 1;
            r_flags = kJobSwap | kJobReadout;
            r_e = e;
            r_ij = ij;
            r_pboff = pbo;
            r_spb = sb;
            r_t1 = T + extra;
          }
          ++inflight;
        }
        if (sdone && inflight == 0) done = true;
      }
      if (done && lane == 0) st.done = 1;
      // ---- the table of the job whose table tick is the next tick
      {
        const int t0 = T + 1 - extra;
        tjob = -1;
        if (t0 >= 0) {
          const int j1 = t0 % D;
          if (rl32(r_valid, j1) && rl32(r_t1, j1) == T + 1) {
            tjob = j1;
            const V4* src = reinterpret_cast<const V4*>(gtab + (size_t)rl32(r_e, j1) * tabw);
            const int nv = tabw / 8;
#pragma unroll
            for (int u = 0; u < kPipeTabVec; ++u) tv[u] = src[min(lane + 64 * u, nv - 1)];
          }
        }
      }
      // ---- the list of the ring rows of the tick after next, layer lp = 2..L in turn
      // and the ring's rows in list order (source 16-byte vector in the planes,
      // destination byte offset in LDS).  Ring lp + 1 of a job lives in pool lp - 1
      // in list order, so only the node ids come from the job's table.  Lane x looks
      // after layer x + 2: one round of header reads, one of node-id reads.
      {
        const int tn = T + 2, pb = tn & 1;
        uint2* rl = reinterpret_cast<uint2*>(smem + pg.off_rows) + pb * pg.rows_max;
        int xj = -1, xt = 0;
        unsigned long long xsrc = 0;
        if (tn - extra - 2 >= 0) {
          const int j2 = (tn - extra - 2) % D;   // slot of the job at layer 2
          for (int x = 0; x + 2 <= Lr; ++x) {
            if (tn - extra - (x + 2) < 0) break;
            const int j = j2 - x < 0 ? j2 - x + D : j2 - x;
            if (!rl32(r_valid, j)) continue;
            const int tbo = rl32(r_tbo, j);
            const unsigned long long src = rl64(r_pboff, j) + (unsigned long long)(Lr + x + 1) * plane;
            if (lane == x) {
              xj = j;
              xt = tbo;
              xsrc = src;
            }
          }
        }
        int xh = 0, xn = 0, xs = 0, xb = 0;
        if (xj >= 0) {
          xh = st.hdr[xj][lane + 2];
          xn = st.hdr[xj][lane + 3] - xh;
          xb = st.rb[xj][lane + 1];
        }
        int nrow = 0;
        for (int x = 0; x + 2 <= Lr; ++x) {
          const int n = rl32(xn, x);
          if (lane == x) xs = nrow;
          nrow += n;
        }
        for (int base = 0; base < nrow; base += 128) {
          int node[2], arow[2];
          unsigned long long src[2];
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const int idx = base + lane + 64 * k;
            int p = 0, tbo = 0, ar = 0;
            unsigned long long s0 = 0;
            for (int x = 0; x + 2 <= Lr; ++x) {
              const int s = rl32(xs, x), n = rl32(xn, x);
              if (idx >= s && idx < s + n) {
                p = rl32(xh, x) + idx - s;
                ar = rl32(xb, x) + idx - s;
                tbo = rl32(xt, x);
                s0 = rl64(xsrc, x);
              }
            }
            node[k] = tabs[tbo + kPipeHdr + p];
            arow[k] = ar;
            src[k] = s0;
          }
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const int idx = base + lane + 64 * k;
            if (idx < nrow)
              rl[idx] = make_uint2((unsigned)((src[k] + (unsigned long long)node[k] * F) / (16 / sizeof(Acc))),
                                   (unsigned)(pg.off_arena + arow[k] * row_bytes));
          }
        }
        if (lane == 0) st.nrows[pb] = nrow;
      }
      copy_load(T);
      __syncthreads();
      if (done) break;
    }
    return;
  }

  // ======================= the compute waves =======================
  // MFMA A fragment of weight block blk (0 message, 1 self), K step stp, output tile tt
  auto afr = [&](int blk, int stp, int tt) { return wl + (((blk * KSB + stp) * MT + tt) * 64 + lane) * VEC; };
  // this lane group's slots of LDS row rw (row and stride fit 24-bit products)
  auto lrow = [&](unsigned rw) {
    return reinterpret_cast<Acc*>(reinterpret_cast<unsigned char*>(arena) + __umul24(rw, (unsigned)row_bytes)) + q * NS;
  };
  // the B operands a tile holds (pipe_to_ops); a lane outside the rows a product
  // computes holds anything: its MFMA column is never used
  using BF = decltype(P::make_b((const Acc*)nullptr));
  auto operands = [&](const Acc (&h)[NS], BF (&bop)[KSB]) { __builtin_memcpy(bop, h, sizeof(BF) * KSB); };

  // a tile's layer input, held across ticks: B operands on the rows computed at the
  // last layer, plain values on the ring rows requested for the next layer until
  // phase B turns them into operands
  Acc hn[MAXT][NS];
#pragma unroll
  for (int k = 0; k < MAXT; ++k)
#pragma unroll
    for (int i = 0; i < NS; ++i) hn[k][i] = (Acc)0;

  // the wave's schedule: lane tau holds its registers' (slot, tile) at ticks tau mod D
  const uint2 my_sched = lane < D ? sched[lane * kMaxWaves + wv] : make_uint2(~0u, ~0u);
  // a tick's tiles (wave-uniform, packed): tk = layer | tile << 8 | slot << 12
  // (layer 0: idle), tb = the job's LDS table, sz = |C_l| | |C_{l+1}| << 16,
  // sm = |C_{l-1}| | message rows (|C_2| at layer 1, else |C_l|) << 16.
  int tk[MAXT], ttb[MAXT], tsz[MAXT], tsm[MAXT];
  int c_nlight = 1, c_rank = 0xff;   // the tick's table conversion: light waves, this wave's rank
  // the same for the next tick, decoded at the start of phase B (the jobs at layers
  // 1..L of the next tick are set up and staged by then) so that its LDS reads
  // complete under the tiles' work
  int nk[MAXT], ntb[MAXT], nsz[MAXT], nsm[MAXT], n_nlight = 1, n_rank = 0xff;
  auto advance = [&]() {
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      tk[k] = nk[k];
      ttb[k] = ntb[k];
      tsz[k] = nsz[k];
      tsm[k] = nsm[k];
    }
    c_nlight = n_nlight;
    c_rank = n_rank;
  };
  auto decode = [&](int tau) {
    const unsigned long long s8 = (unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)my_sched.x, tau) |
                                  ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)my_sched.y, tau) << 32);
    n_nlight = (int)((s8 >> 48) & 0xffu);
    n_rank = (int)(s8 >> 56);
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      const int ent = (int)((s8 >> (8 * k)) & 0xffu);
      nk[k] = 0;
      ntb[k] = nsz[k] = nsm[k] = 0;
      if (ent == 0xff) continue;
      const int j = ent >> 4;
      const int l = (tau - j < 0 ? tau - j + D : tau - j) - extra;
      if (l < 1) continue;
      const int v = st.valid[j], tbo = st.tbo[j];
      const int hm = st.hdr[j][l - 1], h = st.hdr[j][l], hp = st.hdr[j][l + 1], h2 = st.hdr[j][2];
      if (!__builtin_amdgcn_readfirstlane(v)) continue;
      nk[k] = l | (ent & 15) << 8 | j << 12;
      ntb[k] = __builtin_amdgcn_readfirstlane(tbo);
      nsz[k] = __builtin_amdgcn_readfirstlane(h | hp << 16);
      nsm[k] = __builtin_amdgcn_readfirstlane(hm | (l == 1 ? h2 : h) << 16);
    }
  };
  decode(0);
  advance();
  for (int T = 0, tau = 0;; ++T, tau = tau + 1 == D ? 0 : tau + 1) {
    auto tl = [&](int k) { return tk[k] & 0xff; };
    auto tt = [&](int k) { return (tk[k] >> 8) & 15; };
    auto tj = [&](int k) { return tk[k] >> 12; };
    auto tS = [&](int k) { return tsz[k] & 0xffff; };
    auto tSp = [&](int k) { return tsz[k] >> 16; };
    auto tSm = [&](int k) { return tsm[k] & 0xffff; };
    auto tM = [&](int k) { return tsm[k] >> 16; };
    // a phase ends at a barrier, so the waves with the most tiles in it set its
    // length: they issue first (the setup wave above them all)
    int n_a = 0, n_b = 0;
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      n_a += tl(k) >= 1 && tt(k) * 16 < tM(k);
      n_b += tl(k) >= 1 && tt(k) * 16 < tS(k);
    }
    if (n_a >= 2) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(1);
    // ======================= phase A =======================
    // ---- message products G'^{l-1} = H'^{l-1} W_msg of the tiles (into LDS rows);
    // at layer 1 the input is the embedding of the exchanged configuration's spins
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      const int l = tl(k), t = tt(k), j = tj(k);
      if (l < 1 || t * 16 >= tM(k)) continue;
      const uint16_t* tb = tabs + ttb[k];
      const int r = t * 16 + col;
      const bool rin = r < tM(k);
      const int nd = rin ? (int)tb[kPipeHdr + r] : -1;
      if (l == 1) {
        int xs = 0;
        if (rin) {
          const int8_t* sj = sp + j * pg.spw;
          const int2 ij = st.ij[j];
          int8_t v = sj[nd];
          if (st.flags[j] & kJobSwap) v = (nd == ij.x) ? sj[ij.y] : ((nd == ij.y) ? sj[ij.x] : v);
          xs = v > 0 ? 1 : 0;
        }
        lds_read<Acc, NS>(semb + (2 * q + xs) * NS, hn[k]);
      }
      BF bop[KSB];
      operands(hn[k], bop);
      Acc* row = lrow(rin ? tb[kPipeHdr + r8 + r] : 0u);
#pragma unroll
      for (int t4 = 0; t4 < MT; ++t4) {
        CF gs = CF{0, 0, 0, 0};
#pragma unroll
        for (int stp = 0; stp < KSB; ++stp) gs = P::mma(P::load_a(afr(0, stp, t4)), bop[stp], gs);
        Acc gm[4] = {gs[0], gs[1], gs[2], gs[3]};
        if (rin) lds_write<Acc, 4>(row + 4 * t4, gm);
        if (NT == 1024) __builtin_amdgcn_sched_barrier(0);   // one output tile at a time (128 VGPRs)
      }
    }
    // ---- ring rows of this tick -> LDS (requested at the end of the last tick)
    copy_store(T);
    // ---- base H^l of ring l+1 into the lanes of hn that layer l+1 reads from it
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      const int l = tl(k), t = tt(k);
      if (l < 1 || l >= Lr || t * 16 >= tSp(k) || t * 16 + 16 <= tS(k)) continue;
      const int r = t * 16 + col;
      if (r >= tS(k) && r < tSp(k)) {
        const int nd = tabs[ttb[k] + kPipeHdr + r];
        gmem_read<Acc, NS>(planes + st.pboff[tj(k)] + (size_t)(l - 1) * plane + (size_t)nd * F + q * NS, hn[k]);
      }
    }
    // ---- base readout partials of the rows of C_L (tiles at layer L), requested
    // before the barrier (with 16 waves, whose registers are scarce, in phase B,
    // unless phase B stores rows: the sampler)
    constexpr bool kR0Early = NT < 1024 || SWEEP;
    double r0[MAXT][2];
    auto r0_load = [&](int k) {
      r0[k][0] = r0[k][1] = 0.0;
      const int l = tl(k), t = tt(k);
      if (l != Lr || t * 16 >= tS(k) || !(st.flags[tj(k)] & kJobReadout)) return;
      const int r = t * 16 + col;
      if (r < tS(k)) {
        const int nd = tabs[ttb[k] + kPipeHdr + r];
        const double* rp = reinterpret_cast<const double*>(planes + st.pboff[tj(k)] + (size_t)(Lr - 1) * plane) +
                           (size_t)nd * 8 + q * 2;
        r0[k][0] = rp[0];
        r0[k][1] = rp[1];
      }
    };
    if (kR0Early) {
#pragma unroll
      for (int k = 0; k < MAXT; ++k) r0_load(k);
    }
    // ---- sampler: G'^{l-1} changed on C_{l-1}: rows back from LDS into the chain's
    // planes, after this phase's loads (a wait for a load also waits for the stores
    // issued before it)
    if constexpr (SWEEP) {
#pragma unroll
      for (int k = 0; k < MAXT; ++k) {
        const int l = tl(k), t = tt(k);
        if (l < 1 || t * 16 >= tSm(k)) continue;
        const uint16_t* tb = tabs + ttb[k];
        const int r = t * 16 + col;
        if (r < tSm(k)) {
          const int nd = tb[kPipeHdr + r];
          Acc g[NS];
          lds_read<Acc, NS>(lrow(tb[kPipeHdr + r8 + r]), g);
          lds_write<Acc, NS>(planes + st.pboff[tj(k)] + (size_t)(Lr + l - 1) * plane + (size_t)nd * F + q * NS, g);
        }
      }
    }
    __syncthreads();
    if (n_b >= 2) __builtin_amdgcn_s_setprio(2);
    else __builtin_amdgcn_s_setprio(1);
    // ======================= phase B =======================
    // the next tick's ring rows: in flight during this phase (with 16 waves, whose
    // registers are scarce, requested after it)
    if (kR0Early) copy_load(T);
    decode(tau + 1 == D ? 0 : tau + 1);
    double wa = 0.0, wp = 0.0;   // this wave's readout differences of the job at layer L
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
      const int l = tl(k), t = tt(k), j = tj(k);
      if (l < 1) continue;
      if (t * 16 >= tS(k)) {   // no row of C_l: ring rows of layer l + 1 only
        if (l < Lr && t * 16 < tSp(k)) {
          Acc x[NS];
#pragma unroll
          for (int i = 0; i < NS; ++i) x[i] = hn[k][i];
          pipe_to_ops<P, NS>(x, hn[k]);
        }
        continue;
      }
      const uint16_t* tb = tabs + ttb[k];
      const int r = t * 16 + col;
      const bool in = r < tS(k);
      const int nd = in ? (int)tb[kPipeHdr + r] : -1;
      Acc* pw = planes + st.pboff[j];
      const bool last = l == Lr;
      const bool rd = last && (st.flags[j] & kJobReadout);
      if (!kR0Early) r0_load(k);
      // gather sum_d A_hat[n][d] G'^{l-1}[nbr(n, d)] over the job's LDS rows; the sum
      // starts from the first product (a lane outside C_l leaves m unset: never used)
      Acc m[NS];
      if (in) {
        const uint16_t* nbp = tb + kPipeHdr + 2 * r8 + __umul24((unsigned)r, (unsigned)dm);
        const Acc* wpn = sev + __umul24((unsigned)nd, (unsigned)dm);
        auto four = [&](int d, bool first) {
          const uint2 pv = *reinterpret_cast<const uint2*>(nbp + d);
          const unsigned pc[4] = {pv.x & 0xffffu, pv.x >> 16, pv.y & 0xffffu, pv.y >> 16};
          const Acc wt[4] = {wpn[d], wpn[d + 1], wpn[d + 2], wpn[d + 3]};
#pragma unroll
          for (int uu = 0; uu < 4; ++uu) {
            Acc rowv[NS];
            lds_read<Acc, NS>(lrow(pc[uu]), rowv);
            // fused products in neighbour order, as the sum from zero of the full
            // evaluation (written out: contraction may otherwise fuse either product)
#pragma unroll
            for (int i = 0; i < NS; ++i)
              m[i] = __builtin_fmaf(wt[uu], rowv[i], (first && uu == 0) ? 0.0f : m[i]);
            if (NT == 1024) __builtin_amdgcn_sched_barrier(0);   // one neighbour row in flight
          }
        };
        four(0, true);   // dm >= 4
        for (int d = 4; d < dm; d += 4) four(d, false);
      }
      // self product b + H'^{l-1} W_self on the rows of C_l, then the activation
      {
        BF bop[KSB];
        operands(hn[k], bop);
        const Acc* bias = sbias + q * NS;
#pragma unroll
        for (int t4 = 0; t4 < MT; ++t4) {
          CF a;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) a[rr] = bias[4 * t4 + rr];
#pragma unroll
          for (int stp = 0; stp < KSB; ++stp) a = P::mma(P::load_a(afr(1, stp, t4)), bop[stp], a);
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) m[4 * t4 + rr] += a[rr];   // pre-activation (the sum is commutative)
          if (NT == 1024) __builtin_amdgcn_sched_barrier(0);   // one output tile at a time (128 VGPRs)
        }
      }
#pragma unroll
      for (int i = 0; i < NS; ++i) m[i] = P::act(m[i]);
      if (l < Lr) {   // the next layer's input: the rows computed and the ring rows requested
        Acc x[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) x[i] = in ? m[i] : hn[k][i];
        pipe_to_ops<P, NS>(x, hn[k]);
      }
      if (last && (rd || SWEEP)) {   // wave-uniform
        const double* va = shead + q * NS;
        const double* vp = shead + F + q * NS;
        double ta1 = 0, tp1 = 0;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          ta1 += va[i] * (double)m[i];
          tp1 += vp[i] * (double)m[i];
          if (NT == 1024 && i % 4 == 3) __builtin_amdgcn_sched_barrier(0);   // four head weights in flight
        }
        if (rd) {
          double pa = in ? ta1 - r0[k][0] : 0.0;
          double pp = in ? tp1 - r0[k][1] : 0.0;
          wa += wave_sum_dpp(pa);
          wp += wave_sum_dpp(pp);
        }
        if (SWEEP && in) {   // after the base partials were read
          const double rv[2] = {ta1, tp1};
          lds_write<double, 2>(reinterpret_cast<double*>(pw + (size_t)(Lr - 1) * plane) + (size_t)nd * 8 + q * 2, rv);
        }
      } else if (SWEEP && !last && in) {   // H^l changed on C_l
        lds_write<Acc, NS>(pw + (size_t)(l - 1) * plane + (size_t)nd * F + q * NS, m);
      }
    }
    if (lane == 0) {
      red[(T & 1) * 2 * kMaxWaves + wv] = wa;
      red[(T & 1) * 2 * kMaxWaves + kMaxWaves + wv] = wp;
    }
    tab_convert(c_nlight, c_rank);
    advance();
    if (!kR0Early) copy_load(T);
    __syncthreads();
    if (st.done) break;
  }
}

template <class P, int F, int MAXT, int NT, int NCOPY>
__global__ __launch_bounds__(NT) void k_eloc_pipe(Net net, IncNet inc, PipeGeo pg, const uint2* __restrict__ sched,
                                                   const uint16_t* __restrict__ gtab, const int8_t* __restrict__ spins,
                                                   int B, const typename P::Acc* __restrict__ planes, int n_chunks,
                                                   int chunk, double* __restrict__ terms) {
  pipe_body<P, F, MAXT, NT, NCOPY, false>(net, inc, pg, sched, gtab, const_cast<int8_t*>(spins), B,
                                          const_cast<typename P::Acc*>(planes), n_chunks, chunk, terms, 0, 0, 0,
                                          nullptr, nullptr);
}

template <class P, int F, int MAXT, int NT, int NCOPY>
__global__ __launch_bounds__(NT) void k_sweep_pipe(Net net, IncNet inc, PipeGeo pg, const uint2* __restrict__ sched,
                                                    const uint16_t* __restrict__ gtab, int8_t* __restrict__ spins,
                                                    typename P::Acc* planes, int B, int n_sweeps,
                                                    unsigned long long seed, unsigned long long counter_base,
                                                    const unsigned long long* __restrict__ counter_dev,
                                                    int* __restrict__ n_accept) {
  pipe_body<P, F, MAXT, NT, NCOPY, true>(net, inc, pg, sched, gtab, spins, B, planes, 1, 1, nullptr, n_sweeps, seed,
                                         counter_base, counter_dev, n_accept);
}

}  // namespace gna
