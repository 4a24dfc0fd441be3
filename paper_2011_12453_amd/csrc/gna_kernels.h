// Device-side building blocks of the GNA hot path for gfx950: precision traits
// for the MFMA layer products, the Philox4x32-10 generator, and the per-
// configuration evaluator of Eq. 1 shared by the forward, local-energy and
// sampler kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gna {

typedef __attribute__((ext_vector_type(4))) float f4;
typedef __attribute__((ext_vector_type(4))) double d4;
typedef __attribute__((ext_vector_type(4))) short s4;

constexpr int kMaxWaves = 16;           // 1024 threads per workgroup
constexpr int kRowPadBytes = 16;        // LDS row padding of the gather buffer

// ---------------------------------------------------------------------------
// tanh for the FP32/BF16 modes, from its definition tanh(x) = 1 - 2/(exp(2x) + 1).
// The caller passes y = 2 log2(e) x (the factor is folded into the layer's
// weights and bias), so exp(2x) is the hardware base-2 exponential of y.
// Absolute error a few 1e-7; exp overflow gives 1, underflow gives -1.
// ---------------------------------------------------------------------------
constexpr float kTwoLog2e = 2.8853900817779268f;

__device__ __forceinline__ float tanh_from_scaled(float y) {
  const float e = __builtin_amdgcn_exp2f(y);
  return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

typedef __attribute__((ext_vector_type(2))) __bf16 bf2;

// round-to-nearest-even float pair -> packed bfloat16 pair (v_cvt_pk_bf16_f32)
__device__ __forceinline__ unsigned pack_bf16_rne(float a, float b) {
  bf2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(unsigned, v);
}

// ---------------------------------------------------------------------------
// Precision traits.  The layer product of Eq. 1 is computed transposed,
// P^T = W^T [M | H]^T: the MFMA's A operand is W^T (rows = output features),
// its B operand holds 16 nodes (columns) of the activations.  Lane l of a wave
// owns node column l%16 and lane group q = l/16.  Per node tile a lane holds
// F/4 "slots" of features; slot i of lane group q carries logical feature
// lc(q, i), both as an MFMA result and as the next layer's B operand, so the
// activations never leave registers between layers.  row_feature(m) is the
// logical output feature the weight fragment must place in physical A row m
// for that to hold (it follows from each instruction's result layout).
//   Acc: activations, aggregation and accumulation type
//   WT : weight storage type of the A operand
//   BF : B operand built from VEC activations by make_b
//   kScale: factor folded into W and b (act() receives the scaled argument)
// ---------------------------------------------------------------------------
struct PF64 {  // v_mfma_f64_16x16x4f64: D[4r + l/16][l%16], B[l/16][l%16]
  static constexpr int WBLK = 1;   // weight fragment blocks per layer
  using Acc = double;
  using WT = double;
  using AF = double;
  using BF = double;
  using CF = d4;
  static constexpr int KS = 4, VEC = 1;
  static constexpr double kScale = 1.0;
  __device__ static BF make_b(const Acc* x) { return x[0]; }
  __device__ static AF load_a(const WT* p) { return p[0]; }
  __device__ static CF mma(const AF& a, const BF& b, CF c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static constexpr int NPART = 1;
  __device__ static CF mma_part(const AF& a, const BF& b, int, CF c) { return mma(a, b, c); }
  __host__ __device__ static int lc(int q, int i) { return 4 * i + q; }
  __host__ __device__ static int row_feature(int m) { return m; }
  __device__ static WT to_w(double v) { return v; }
  __device__ static Acc act(Acc x) { return tanh(x); }
};

struct PF32 {  // v_mfma_f32_16x16x4f32: D[4(l/16) + r][l%16], B[l/16][l%16]
  static constexpr int WBLK = 1;   // weight fragment blocks per layer
  using Acc = float;
  using WT = float;
  using AF = float;
  using BF = float;
  using CF = f4;
  static constexpr int KS = 4, VEC = 1;
  static constexpr double kScale = (double)kTwoLog2e;
  __device__ static BF make_b(const Acc* x) { return x[0]; }
  __device__ static AF load_a(const WT* p) { return p[0]; }
  __device__ static CF mma(const AF& a, const BF& b, CF c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static constexpr int NPART = 1;
  __device__ static CF mma_part(const AF& a, const BF& b, int, CF c) { return mma(a, b, c); }
  __host__ __device__ static int lc(int q, int i) { return 4 * i + q; }
  __host__ __device__ static int row_feature(int m) {
    return 16 * (m / 16) + 4 * (m % 4) + (m % 16) / 4;
  }
  __device__ static WT to_w(double v) { return (float)v; }
  __device__ static Acc act(Acc y) { return tanh_from_scaled(y); }
};

// BF16 operands.  Weights are rounded to bfloat16 once.  Each activation x is
// carried as the unevaluated pair hi + lo of two bfloat16 values (hi = x with its
// low 16 bits cleared, lo = RNE(x - hi)), i.e. about 16 significant bits, and
// every product is issued as two MFMAs, W.hi + W.lo, accumulated in FP32.
struct PBF16 {  // v_mfma_f32_16x16x16_bf16: D[4(l/16) + r][l%16], B[4(l/16) + j][l%16]
  static constexpr int WBLK = 1;   // weight fragment blocks per layer
  using Acc = float;
  using WT = unsigned short;  // bfloat16 bits
  struct BF { s4 hi, lo; };
  using CF = f4;
  static constexpr int KS = 16, VEC = 4;
  static constexpr double kScale = (double)kTwoLog2e;
  __device__ static BF make_b(const Acc* x) {
    unsigned u[4];
    float r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      u[j] = __float_as_uint(x[j]) & 0xFFFF0000u;
      r[j] = x[j] - __uint_as_float(u[j]);
    }
    BF b;
    const unsigned h01 = (u[0] >> 16) | u[1], h23 = (u[2] >> 16) | u[3];
    const unsigned l01 = pack_bf16_rne(r[0], r[1]), l23 = pack_bf16_rne(r[2], r[3]);
    b.hi = __builtin_bit_cast(s4, (unsigned long long)h01 | ((unsigned long long)h23 << 32));
    b.lo = __builtin_bit_cast(s4, (unsigned long long)l01 | ((unsigned long long)l23 << 32));
    return b;
  }
  using AF = s4;
  __device__ static AF load_a(const WT* p) { return *reinterpret_cast<const s4*>(p); }
  __device__ static CF mma(const AF& a, const BF& b, CF c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b.hi, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b.lo, c, 0, 0, 0);
  }
  static constexpr int NPART = 2;   // hi, then lo
  __device__ static CF mma_part(const AF& a, const BF& b, int part, CF c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, part ? b.lo : b.hi, c, 0, 0, 0);
  }
  __host__ __device__ static int lc(int q, int i) { return 16 * (i / 4) + 4 * q + (i % 4); }
  __host__ __device__ static int row_feature(int m) { return m; }
  __device__ static WT to_w(double v) {
    return (WT)(pack_bf16_rne((float)v, 0.0f) & 0xFFFFu);
  }
  __device__ static Acc act(Acc y) { return tanh_from_scaled(y); }
};

// The same operands on v_mfma_f32_16x16x32_bf16 (F a multiple of 32):
// B[8(l/16) + j][l%16], j = 0..7, so slot i of lane group q is feature
// 32(i/8) + 8q + i%8, and physical A row 16t + 4q + r must compute that
// feature of slot 4t + r.
typedef __attribute__((ext_vector_type(8))) __bf16 bf8v;
struct PBF16W {
  static constexpr int WBLK = 1;   // weight fragment blocks per layer
  using Acc = float;
  using WT = unsigned short;
  struct BF { bf8v hi, lo; };
  using CF = f4;
  static constexpr int KS = 32, VEC = 8;
  static constexpr double kScale = (double)kTwoLog2e;
  __device__ static BF make_b(const Acc* x) {
    unsigned hu[4], lu[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const unsigned u0 = __float_as_uint(x[2 * p]) & 0xFFFF0000u;
      const unsigned u1 = __float_as_uint(x[2 * p + 1]) & 0xFFFF0000u;
      hu[p] = (u0 >> 16) | u1;
      lu[p] = pack_bf16_rne(x[2 * p] - __uint_as_float(u0), x[2 * p + 1] - __uint_as_float(u1));
    }
    BF b;
    b.hi = __builtin_bit_cast(bf8v, uint4{hu[0], hu[1], hu[2], hu[3]});
    b.lo = __builtin_bit_cast(bf8v, uint4{lu[0], lu[1], lu[2], lu[3]});
    return b;
  }
  using AF = bf8v;
  __device__ static AF load_a(const WT* p) { return *reinterpret_cast<const bf8v*>(p); }
  __device__ static CF mma(const AF& a, const BF& b, CF c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.hi, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.lo, c, 0, 0, 0);
  }
  static constexpr int NPART = 2;   // hi, then lo
  __device__ static CF mma_part(const AF& a, const BF& b, int part, CF c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, part ? b.lo : b.hi, c, 0, 0, 0);
  }
  __host__ __device__ static int lc(int q, int i) { return 32 * (i / 8) + 8 * q + (i % 8); }
  __host__ __device__ static int row_feature(int m) {
    const int t = m / 16, q = (m % 16) / 4, r = m % 4;
    return 32 * (t / 2) + 8 * q + 4 * (t % 2) + r;
  }
  __device__ static WT to_w(double v) {
    return (WT)(pack_bf16_rne((float)v, 0.0f) & 0xFFFFu);
  }
  __device__ static Acc act(Acc y) { return tanh_from_scaled(y); }
};

// Single-pass BF16: the activations are rounded to the nearest bfloat16 and each
// product is one MFMA (the classic BF16 operand precision; about 8 significant
// bits per operand instead of the split pair's 16).  Same layouts as above.
struct PBF161 : PBF16 {
  using BF = s4;
  static constexpr int NPART = 1;
  __device__ static BF make_b(const Acc* x) {
    const unsigned l01 = pack_bf16_rne(x[0], x[1]), l23 = pack_bf16_rne(x[2], x[3]);
    return __builtin_bit_cast(s4, (unsigned long long)l01 | ((unsigned long long)l23 << 32));
  }
  __device__ static CF mma(const AF& a, const BF& b, CF c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
  __device__ static CF mma_part(const AF& a, const BF& b, int, CF c) { return mma(a, b, c); }
};

// Split BF16 weights as well as activations, for ReLU + layer normalisation (whose
// normalised layers carry the 8-bit rounding of bfloat16 weights to the output at
// unit scale): each weight is the pair hi + lo of bfloat16 values (hi = RNE(w),
// lo = RNE(w - hi)), and every product is issued as three MFMAs, hi x hi, hi x lo
// and lo x hi (lo x lo is below the FP32 accumulation's rounding).  A layer's block
// of weight fragments holds the hi fragments, then the lo fragments (2 F^2 each).
template <int F_>
struct PBF16S : PBF16W {
  static constexpr int WBLK = 2;
  struct AF { bf8v hi, lo; };
  __device__ static AF load_a(const WT* p) {
    AF a;
    a.hi = *reinterpret_cast<const bf8v*>(p);
    a.lo = *reinterpret_cast<const bf8v*>(p + 2 * F_ * F_);
    return a;
  }
  __device__ static CF mma(const AF& a, const BF& b, CF c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, c, 0, 0, 0);
  }
  static constexpr int NPART = 3;   // hi x hi, hi x lo, lo x hi
  __device__ static CF mma_part(const AF& a, const BF& b, int part, CF c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(part == 2 ? a.lo : a.hi, part == 1 ? b.lo : b.hi, c, 0, 0, 0);
  }
  __device__ static WT to_w_lo(double v) {
    const unsigned h = pack_bf16_rne((float)v, 0.0f) & 0xFFFFu;
    const double hv = (double)__uint_as_float(h << 16);
    return (WT)(pack_bf16_rne((float)(v - hv), 0.0f) & 0xFFFFu);
  }
};

struct PBF16W1 : PBF16W {
  using BF = bf8v;
  static constexpr int NPART = 1;
  __device__ static BF make_b(const Acc* x) {
    unsigned u[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) u[p] = pack_bf16_rne(x[2 * p], x[2 * p + 1]);
    return __builtin_bit_cast(bf8v, uint4{u[0], u[1], u[2], u[3]});
  }
  __device__ static CF mma(const AF& a, const BF& b, CF c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static CF mma_part(const AF& a, const BF& b, int, CF c) { return mma(a, b, c); }
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products,
// XOR recombination with the key, key advanced by Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}

// ---------------------------------------------------------------------------
// Launch geometry and LDS layout (byte offsets into dynamic shared memory).
// ---------------------------------------------------------------------------
struct Geo {
  int wpc;        // waves per workgroup; the workgroup evaluates one configuration
  int ntiles;     // node tiles: wpc * TPW >= ceil(N / 16), every wave owns TPW of them
  int npad;       // 16 * ntiles (nodes past N are padding with zero adjacency)
  int nbuf;       // 1 or 2 gather buffers
  int row_elems;  // gather-buffer row stride in elements of Acc
  int buf_elems;  // elements of Acc per gather buffer
  int off_w, off_h, off_sp, off_idx, off_val, off_red;
  int off_bias, off_emb, off_head;   // layer biases [nW][F], embedding [2][F], heads [2][F+3]
  int lds_bytes;
};

struct Net {
  int n, ne, F, L, tied, dmax;
  int act;                 // 0: tanh (weights pre-scaled by kScale); 1: ReLU + layer normalisation (unscaled)
  const int* ell_idx;      // [npad][dmax] neighbour ids (padding points at the node itself)
  const void* ell_val;     // [npad][dmax] A_hat values in Acc precision (padding 0)
  const int2* edges;       // [ne] bond endpoints
  const void* wfrag;       // [nW][2F/KS][F/16][64][VEC] weight fragments, WT (scaled by kScale)
  const void* bias;        // [nW][F] logical order, Acc (scaled by kScale)
  const void* emb;         // [2][F] tanh(W_e[x] + b_e), Acc, logical order
  const double* head_a;    // v_a[F+2], c_a (FP64, inside theta)
  const double* head_p;    // v_p[F+2], c_p
  Geo g;
};

// FP64 wavefront sum through DPP lane moves (no LDS traffic), fixed order; the
// total is returned to every lane.  Steps: pairs and quads (quad_perm), halves
// of a row (row_half_mirror), rows of 16 (row_mirror), then row 0 -> 1 and
// row 2 -> 3 (row_bcast:15) and rows 0-1 -> 2-3 (row_bcast:31); lane 63 holds
// the sum.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xb1>(v);          // quad_perm(1,0,3,2)
  v += dpp_f64<0x4e>(v);          // quad_perm(2,3,0,1)
  v += dpp_f64<0x141>(v);         // row_half_mirror
  v += dpp_f64<0x140>(v);         // row_mirror
  v += dpp_f64<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, 63), hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// fixed-order FP64 wavefront sum (same order for every configuration)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// ReLU followed by a layer normalisation over a node's F features (the paper's f,
// Section 2).  The node's features sit in the 4 lanes q = 0..3 of its column (NS
// slots each); row sums go through a fixed butterfly (lane xor 16, then xor 32),
// so all four lanes, and every evaluation of the same row, get identical values.
// ---------------------------------------------------------------------------
constexpr double kLnEps = 1e-5;

template <class Acc>
__device__ __forceinline__ Acc quad_sum(Acc v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// y = ReLU(x); mean and inverse standard deviation of y over the row
template <class Acc, int NS>
__device__ __forceinline__ void relu_ln_stats(const Acc (&x)[NS], Acc (&y)[NS], Acc& mu, Acc& r) {
  constexpr int F = 4 * NS;
  Acc s = 0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    y[i] = x[i] > (Acc)0 ? x[i] : (Acc)0;
    s += y[i];
  }
  mu = quad_sum(s) / (Acc)F;
  Acc v = 0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const Acc d = y[i] - mu;
    v += d * d;
  }
  r = (Acc)1 / sqrt(quad_sum(v) / (Acc)F + (Acc)kLnEps);
}

template <class Acc, int NS>
__device__ __forceinline__ void relu_ln_row(const Acc (&x)[NS], Acc (&y)[NS], Acc (&h)[NS]) {
  Acc mu, r;
  relu_ln_stats<Acc, NS>(x, y, mu, r);
#pragma unroll
  for (int i = 0; i < NS; ++i) h[i] = (y[i] - mu) * r;
}

// cotangent of the pre-activation from that of h = LN(ReLU(x)), given y = ReLU(x)
// and h: dy = r (dh - mean dh - h mean(dh h)), dx = dy [y > 0]
template <class Acc, int NS>
__device__ __forceinline__ void relu_ln_vjp(const Acc (&y)[NS], const Acc (&h)[NS], const Acc (&dh)[NS],
                                            Acc (&dx)[NS]) {
  constexpr int F = 4 * NS;
  Acc yy[NS], mu, r;
  relu_ln_stats<Acc, NS>(y, yy, mu, r);   // ReLU of y is y
  Acc a = 0, b = 0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    a += dh[i];
    b += dh[i] * h[i];
  }
  const Acc ma = quad_sum(a) / (Acc)F, mb = quad_sum(b) / (Acc)F;
#pragma unroll
  for (int i = 0; i < NS; ++i) dx[i] = y[i] > (Acc)0 ? r * (dh[i] - ma - h[i] * mb) : (Acc)0;
}

// vectorised LDS copy of N elements of T (alignment 16 B or of the chunk size)
template <class T, int N>
__device__ __forceinline__ void lds_read(const T* __restrict__ src, T (&dst)[N]) {
  constexpr int B = N * (int)sizeof(T);
  if constexpr (B % 16 == 0) {
    const uint4* s = reinterpret_cast<const uint4*>(src);
#pragma unroll
    for (int k = 0; k < B / 16; ++k) reinterpret_cast<uint4*>(dst)[k] = s[k];
  } else if constexpr (B % 8 == 0) {
    const uint2* s = reinterpret_cast<const uint2*>(src);
#pragma unroll
    for (int k = 0; k < B / 8; ++k) reinterpret_cast<uint2*>(dst)[k] = s[k];
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) dst[k] = src[k];
  }
}
template <class T, int N>
__device__ __forceinline__ void lds_write(T* __restrict__ dst, const T* src) {
  constexpr int B = N * (int)sizeof(T);
  if constexpr (B % 16 == 0) {
#pragma unroll
    for (int k = 0; k < B / 16; ++k)
      reinterpret_cast<uint4*>(dst)[k] = reinterpret_cast<const uint4*>(src)[k];
  } else if constexpr (B % 8 == 0) {
#pragma unroll
    for (int k = 0; k < B / 8; ++k)
      reinterpret_cast<uint2*>(dst)[k] = reinterpret_cast<const uint2*>(src)[k];
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) dst[k] = src[k];
  }
}

// copy of N elements of T from global memory (16-byte aligned rows), issued as
// global loads, so that a branch between an LDS row and a global row is never
// merged into one flat access
template <class T, int N>
__device__ __forceinline__ void gmem_read(const T* src, T (&dst)[N]) {
  constexpr int B = N * (int)sizeof(T);
  static_assert(B % 16 == 0, "rows are whole 16-byte vectors");
  using V = unsigned int __attribute__((ext_vector_type(4)));
  using G = const __attribute__((address_space(1))) V*;
  G s = (G)(src);
#pragma unroll
  for (int k = 0; k < B / 16; ++k) reinterpret_cast<V*>(dst)[k] = s[k];
}

// ---------------------------------------------------------------------------
// Per-workgroup view of LDS.
// ---------------------------------------------------------------------------
template <class P>
struct Smem {
  using WT = typename P::WT;
  using Acc = typename P::Acc;
  WT* w;         // one layer's weight fragments
  Acc* h;        // gather buffer(s)
  int8_t* sp;    // spins of the current sample
  int* idx;      // ELL neighbour ids
  Acc* val;      // ELL values
  double* red;   // [2 * kMaxWaves] readout partials + scalars
  Acc* bias;     // [nW][4][F/4]: layer bias in slot order, lane group q at q*F/4
  Acc* emb;      // [2][F]
  double* head;  // v_a[F+2], c_a, v_p[F+2], c_p
  __device__ Smem(const Geo& g, unsigned char* base)
      : w(reinterpret_cast<WT*>(base + g.off_w)),
        h(reinterpret_cast<Acc*>(base + g.off_h)),
        sp(reinterpret_cast<int8_t*>(base + g.off_sp)),
        idx(reinterpret_cast<int*>(base + g.off_idx)),
        val(reinterpret_cast<Acc*>(base + g.off_val)),
        red(reinterpret_cast<double*>(base + g.off_red)),
        bias(reinterpret_cast<Acc*>(base + g.off_bias)),
        emb(reinterpret_cast<Acc*>(base + g.off_emb)),
        head(reinterpret_cast<double*>(base + g.off_head)) {}
};

// red[] scalar slots after the 2*kMaxWaves partials
constexpr int kRedNup = 2 * kMaxWaves;      // number of up spins (as double)
constexpr int kRedFlag = 2 * kMaxWaves + 1; // sampler accept flag / broadcast
constexpr int kRedSlots = 2 * kMaxWaves + 4;

// Copy one layer's weight fragments global -> LDS (whole workgroup).
template <class P, int F>
__device__ void stage_weights(const Net& net, const Smem<P>& s, int layer) {
  using WT = typename P::WT;
  constexpr int n = P::WBLK * 2 * F * F;  // elements per layer
  const WT* src = reinterpret_cast<const WT*>(net.wfrag) + (size_t)layer * n;
  if constexpr ((n * sizeof(WT)) % 16 == 0) {
    const uint4* s4p = reinterpret_cast<const uint4*>(src);
    uint4* d4p = reinterpret_cast<uint4*>(s.w);
    for (int k = threadIdx.x; k < (int)(n * sizeof(WT) / 16); k += blockDim.x) d4p[k] = s4p[k];
  } else {
    for (int k = threadIdx.x; k < n; k += blockDim.x) s.w[k] = src[k];
  }
}

// Copy the ELL adjacency, the biases, the embedding table and the head weights
// global -> LDS (whole workgroup).
template <class P>
__device__ void stage_graph(const Net& net, const Smem<P>& s) {
  using Acc = typename P::Acc;
  const int n = net.g.npad * net.dmax;
  const Acc* v = reinterpret_cast<const Acc*>(net.ell_val);
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    s.idx[k] = net.ell_idx[k];
    s.val[k] = v[k];
  }
  const int nb = (net.tied ? 1 : net.L) * net.F;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    const int lay = k / net.F, e = k % net.F, qq = e / (net.F / 4), i = e % (net.F / 4);
    s.bias[k] = reinterpret_cast<const Acc*>(net.bias)[lay * net.F + P::lc(qq, i)];
  }
  for (int k = threadIdx.x; k < 2 * net.F; k += blockDim.x) s.emb[k] = reinterpret_cast<const Acc*>(net.emb)[k];
  for (int k = threadIdx.x; k < net.F + 3; k += blockDim.x) {
    s.head[k] = net.head_a[k];
    s.head[net.F + 3 + k] = net.head_p[k];
  }
}

// Load one sample's spins into LDS and count its up spins into red[kRedNup].
// Ends with a barrier.
template <class P>
__device__ void load_spins(const Net& net, const Smem<P>& s, const int8_t* __restrict__ src) {
  __shared__ int nup;
  if (threadIdx.x == 0) nup = 0;
  __syncthreads();
  int c = 0;
  for (int k = threadIdx.x; k < net.g.npad; k += blockDim.x) {
    const int8_t v = (k < net.n) ? src[k] : (int8_t)-1;
    s.sp[k] = v;
    c += (k < net.n && v > 0) ? 1 : 0;
  }
  if (c) atomicAdd(&nup, c);
  __syncthreads();
  if (threadIdx.x == 0) s.red[kRedNup] = (double)nup;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Evaluate log psi of the configuration in s.sp with sites si and sj exchanged
// (si < 0: no exchange).  Whole workgroup; the result is returned to thread 0
// only.  Node tile k of wave w is tile w + k * wpc.
//
// Eq. 1 is applied as P = A_hat (H W_msg) + H W_self + b: both products take the
// node's own activations as the MFMA B operand (built once per tile), the
// message product G = H W_msg goes through LDS, and the adjacency gather adds
// A_hat G into the accumulator before tanh.  The message product is split into
// NCH chunks of output features when the LDS buffer must be smaller.
//
// Every call performs the same arithmetic in the same order for a node whose
// receptive field holds the same spins, so log psi differences cancel exactly
// outside it.
//   STORE == 1: also write the layer inputs H^0..H^L and messages M^0..M^{L-1}
//   (M^l = A_hat H^l, gathered for the reverse pass) to `store` as planes of
//   npad x F values, element (node, q, i) at node * F + q * F/4 + i (slot
//   order); H^l is plane l, M^l plane L + 1 + l; with ReLU + layer normalisation
//   also the post-ReLU rows Y^l (l = 1..L) as planes 2L + 4 + l.
//   STORE == 2: write the base planes of the incremental local energy: layer
//   outputs H^1..H^{L-1} as planes 0..L-2, the layer-L readout partials (per
//   node and lane quad q, the pair (t_a, t_p) of FP64 sums v . H^L over the
//   quad's slots) in plane L-1 as doubles at node * 8 + q * 2, and message
//   products G^l = H^l W_msg (l = 0..L-1) as planes L..2L-1, same element order.
// ---------------------------------------------------------------------------
template <class P, int F, int TPW, int NCH, int STORE = 0>
__device__ void eval_config(const Net& net, const Smem<P>& s, int si, int sj,
                            double& out_la, double& out_ph,
                            typename P::Acc* __restrict__ store = nullptr) {
  using Acc = typename P::Acc;
  using WT = typename P::WT;
  using AF = typename P::AF;
  using BF = typename P::BF;
  using CF = typename P::CF;
  constexpr int NS = F / 4;           // slots per lane per tile
  constexpr int MT = F / 16;          // output 16-feature tiles
  constexpr int KSB = F / P::KS;      // MFMA k-steps per F-wide block
  constexpr int MTC = MT / NCH;       // output tiles per message chunk
  constexpr int CS = NS / NCH;        // slots per message chunk
  constexpr int VEC = P::VEC;
  static_assert(F % 16 == 0 && KSB >= 1 && MT % NCH == 0, "bad shape");

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int q = lane >> 4, col = lane & 15;
  const Geo& g = net.g;
  const int wpc = g.wpc;

  int node[TPW];
  bool tile_ok[TPW], real[TPW];
  Acc h[TPW][NS];
  const Acc* emb = s.emb;
  const double* head_a = s.head;
  const double* head_p = s.head + F + 3;
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int tile = wv + k * wpc;
    tile_ok[k] = true;   // ntiles == wpc * TPW: every tile slot holds a tile
    node[k] = tile * 16 + col;
    real[k] = tile_ok[k] && node[k] < net.n;
    int x = 0;
    if (real[k]) {
      const int nd = node[k];
      const int8_t sv = (nd == si) ? s.sp[sj] : ((nd == sj) ? s.sp[si] : s.sp[nd]);
      x = sv > 0 ? 1 : 0;
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) h[k][i] = real[k] ? emb[x * F + P::lc(q, i)] : (Acc)0;
  }

  double pa = 0.0, pp = 0.0;
  const WT* wl = s.w;
  const size_t plane = (size_t)g.npad * F;
  // weight fragment of output tile t at k-step st of block blk (0 message, 1 self)
  auto afrag = [&](int blk, int st, int t) { return wl + (((blk * KSB + st) * MT + t) * 64 + lane) * VEC; };
  for (int l = 0; l < net.L; ++l) {
    if constexpr (STORE == 1) {
#pragma unroll
      for (int k = 0; k < TPW; ++k)
        if (tile_ok[k]) lds_write<Acc, NS>(store + l * plane + node[k] * F + q * NS, h[k]);
    }
    if (!net.tied) {
      __syncthreads();
      stage_weights<P, F>(net, s, l);
      __syncthreads();
    }
    const Acc* bias = s.bias + (net.tied ? 0 : l) * F + q * NS;   // this lane group's slots
    // B operands of every tile of the wave, built once per layer (BF16 types
    // only; FP32/FP64 operands are the activations themselves)
    constexpr bool SPLIT = (P::VEC > 1);   // multi-element (BF16) fragments
    BF bfr[SPLIT ? TPW : 1][SPLIT ? KSB : 1];
    if constexpr (SPLIT) {
#pragma unroll
      for (int k = 0; k < TPW; ++k)
#pragma unroll
        for (int st = 0; st < KSB; ++st) bfr[k][st] = P::make_b(&h[k][st * VEC]);
    }
    auto bop = [&](int k, int st) -> BF {
      if constexpr (SPLIT) return bfr[k][st];
      else return P::make_b(&h[k][st * VEC]);
    };
    CF acc[TPW][MT];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const int buf = (g.nbuf == 2) ? ((l * NCH + ch) & 1) : 0;
      Acc* hb = s.h + buf * g.buf_elems;
      if (g.nbuf == 1) __syncthreads();           // the previous gather is done
      if constexpr (SPLIT) {
      // Output tiles outermost: each weight fragment is read once and applied to
      // every tile; the hi and lo halves of a product are issued tile after tile.
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const bool self_t = (ch == 0);            // self product once, in the first chunk
        const bool msg_t = (t / MTC == ch);       // message product of this chunk's tiles
        if (self_t) {
          CF bt;
#pragma unroll
          for (int r = 0; r < 4; ++r) bt[r] = bias[4 * t + r];
#pragma unroll
          for (int st = 0; st < KSB; ++st) {
            const AF a = P::load_a(afrag(1, st, t));
#pragma unroll
            for (int part = 0; part < P::NPART; ++part)
#pragma unroll
              for (int k = 0; k < TPW; ++k)
                if (tile_ok[k])
                  acc[k][t] = P::mma_part(a, bop(k, st), part, (st == 0 && part == 0) ? bt : acc[k][t]);
          }
        }
        if (msg_t) {
          CF gacc[TPW];
#pragma unroll
          for (int st = 0; st < KSB; ++st) {
            const AF a = P::load_a(afrag(0, st, t));
#pragma unroll
            for (int part = 0; part < P::NPART; ++part)
#pragma unroll
              for (int k = 0; k < TPW; ++k)
                if (tile_ok[k])
                  gacc[k] = P::mma_part(a, bop(k, st), part, (st == 0 && part == 0) ? CF{0, 0, 0, 0} : gacc[k]);
          }
#pragma unroll
          for (int k = 0; k < TPW; ++k)
            if (tile_ok[k]) {
              Acc gm[4] = {gacc[k][0], gacc[k][1], gacc[k][2], gacc[k][3]};
              lds_write<Acc, 4>(hb + node[k] * g.row_elems + q * CS + 4 * (t - ch * MTC), gm);
              if constexpr (STORE == 2)
                lds_write<Acc, 4>(store + (net.L + l) * plane + node[k] * F + q * NS + 4 * t, gm);
            }
        }
      }
      } else {
      // one-word fragments: tiles outermost keeps the live set small
#pragma unroll
      for (int k = 0; k < TPW; ++k) {
        if (!tile_ok[k]) continue;
        if (ch == 0) {
#pragma unroll
          for (int t = 0; t < MT; ++t) {
            CF a;
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = bias[4 * t + r];
#pragma unroll
            for (int st = 0; st < KSB; ++st) a = P::mma(P::load_a(afrag(1, st, t)), bop(k, st), a);
            acc[k][t] = a;
          }
        }
        Acc gm[CS];
#pragma unroll
        for (int tc = 0; tc < MTC; ++tc) {
          CF a = CF{0, 0, 0, 0};
#pragma unroll
          for (int st = 0; st < KSB; ++st) a = P::mma(P::load_a(afrag(0, st, ch * MTC + tc)), bop(k, st), a);
#pragma unroll
          for (int r = 0; r < 4; ++r) gm[4 * tc + r] = a[r];
        }
        lds_write<Acc, CS>(hb + node[k] * g.row_elems + q * CS, gm);
        if constexpr (STORE == 2)
          lds_write<Acc, CS>(store + (net.L + l) * plane + node[k] * F + q * NS + ch * CS, gm);
      }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < TPW; ++k) {
        if (!tile_ok[k]) continue;
        const int* ip = s.idx + node[k] * net.dmax;
        const Acc* vp = s.val + node[k] * net.dmax;
        Acc m[CS];
#pragma unroll
        for (int i = 0; i < CS; ++i) m[i] = (Acc)0;
        // the neighbour list is padded to a multiple of 4 (zero weights); degree-4
        // graphs (Kagome) take the straight-line path
        auto gather4 = [&](int d) {
          Acc row[4][CS];
#pragma unroll
          for (int u = 0; u < 4; ++u) lds_read<Acc, CS>(hb + ip[d + u] * g.row_elems + q * CS, row[u]);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const Acc a = vp[d + u];
#pragma unroll
            for (int i = 0; i < CS; ++i) m[i] += a * row[u][i];
          }
        };
        if (net.dmax == 4) {
          gather4(0);
        } else {
          for (int d = 0; d < net.dmax; d += 4) gather4(d);
        }
#pragma unroll
        for (int tc = 0; tc < MTC; ++tc)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[k][ch * MTC + tc][r] += m[4 * tc + r];
      }
    }
    if constexpr (STORE == 1) {
      // the reverse pass needs M^l = A_hat H^l itself: gather H^l (one more LDS round)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        const int buf = (g.nbuf == 2) ? ((l * NCH + ch + 1) & 1) : 0;
        Acc* hb = s.h + buf * g.buf_elems;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < TPW; ++k)
          if (tile_ok[k]) lds_write<Acc, CS>(hb + node[k] * g.row_elems + q * CS, &h[k][ch * CS]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < TPW; ++k) {
          if (!tile_ok[k]) continue;
          Acc m[CS];
#pragma unroll
          for (int i = 0; i < CS; ++i) m[i] = (Acc)0;
          // in neighbour order, four rows requested at a time (the list is padded to a
          // multiple of 4)
          for (int d = 0; d < net.dmax; d += 4) {
            Acc row[4][CS];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              lds_read<Acc, CS>(hb + s.idx[node[k] * net.dmax + d + u] * g.row_elems + q * CS, row[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const Acc a = s.val[node[k] * net.dmax + d + u];
#pragma unroll
              for (int i = 0; i < CS; ++i) m[i] += a * row[u][i];
            }
          }
          lds_write<Acc, CS>(store + (net.L + 1 + l) * plane + node[k] * F + q * NS + ch * CS, m);
        }
      }
      __syncthreads();
    }
    const bool last = (l == net.L - 1);
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
      // readout partial of this node (its lane group's slots) in FP64: identical
      // inputs give identical partials, so unchanged nodes still cancel exactly in
      // log psi differences
      double ta = 0, tp = 0;
      if (net.act == 0) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const Acc v = P::act(acc[k][t][r]);
            h[k][4 * t + r] = v;
          }
        }
      } else {
        Acc pre[NS], y[NS];
#pragma unroll
        for (int t = 0; t < MT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) pre[4 * t + r] = acc[k][t][r];
        relu_ln_row<Acc, NS>(pre, y, h[k]);
        if constexpr (STORE == 1) {
          if (tile_ok[k]) lds_write<Acc, NS>(store + (2 * net.L + 5 + l) * plane + node[k] * F + q * NS, y);
        }
      }
      if (last) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const int f = P::lc(q, i);
          ta += head_a[f] * (double)h[k][i];
          tp += head_p[f] * (double)h[k][i];
        }
      }
      if (last && real[k]) {
        pa += ta;
        pp += tp;
      }
      if constexpr (STORE == 2) {
        if (!last) {
          lds_write<Acc, NS>(store + l * plane + node[k] * F + q * NS, h[k]);
        } else if (tile_ok[k]) {   // layer L: the node's FP64 readout partials, not its row
          const double rv[2] = {ta, tp};
          lds_write<double, 2>(reinterpret_cast<double*>(store + l * plane) + node[k] * 8 + q * 2, rv);
        }
      }
    }
  }
  if constexpr (STORE == 1) {
#pragma unroll
    for (int k = 0; k < TPW; ++k)
      if (tile_ok[k]) lds_write<Acc, NS>(store + net.L * plane + node[k] * F + q * NS, h[k]);
  }
  if (net.L == 0) {
#pragma unroll
    for (int k = 0; k < TPW; ++k)
      if (real[k])
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          const int f = P::lc(q, i);
          pa += head_a[f] * (double)h[k][i];
          pp += head_p[f] * (double)h[k][i];
        }
  }
  pa = wave_sum(pa);
  pp = wave_sum(pp);
  if (lane == 0) {
    s.red[wv] = pa;
    s.red[kMaxWaves + wv] = pp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, p = 0.0;
    for (int w = 0; w < wpc; ++w) {
      a += s.red[w];
      p += s.red[kMaxWaves + w];
    }
    const double nup = s.red[kRedNup], ndn = (double)net.n - nup;
    a += head_a[F] * ndn + head_a[F + 1] * nup + head_a[F + 2];
    p += head_p[F] * ndn + head_p[F + 1] * nup + head_p[F + 2];
    out_la = a;
    out_ph = p;
  }
  __syncthreads();
}

}  // namespace gna
