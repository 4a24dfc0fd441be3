/*
 * gna.h - C ABI of the graph-neural-ansatz variational Monte Carlo hot path on
 * AMD Instinct MI355X (gfx950).
 *
 * What the library computes (the paper: "Scalable variational Monte Carlo with
 * graph neural ansatz", Yang, Hu, Li; NeurIPS 2020 ML4PS workshop):
 *
 *   ansatz (Section 2, Eq. 1):  H0_i = f(onehot(x_i) W_e + b_e),
 *        H^{l+1} = f([A_hat H^l ; H^l] W + b),  A_hat = D^-1/2 A D^-1/2,
 *        z = sum_i [H^L_i ; onehot(x_i)],  log psi = (v_a.z + c_a) + i (v_p.z + c_p)
 *        (the two-head complex form the paper names in Section 5), with f = tanh
 *        or the paper's ReLU followed by a layer normalisation (config field
 *        activation);
 *   local energy (Section 3, E_x = sum_x' H_xx' Psi_x'/Psi_x) of the spin-1/2
 *        Heisenberg model:  E(s) = sum_<ij> [Jz s_i s_j/4
 *                                 + (Jxy/2)[s_i != s_j] psi(s^ij)/psi(s)],
 *        or any bond Hamiltonian of that form with a field and a constant per
 *        bond, which covers the hard-core bosons of Eq. 4 (gna_set_couplings);
 *   Metropolis spin-swap sampling of |psi|^2 (Section 3), and the grouping of
 *        duplicated samples into unique states with counts (Section 3);
 *   ISGO gradient (Section 3, Eq. 3): samples drawn under psi_old reused with
 *        self-normalised weights p_x ~ n_x |psi_x|^2 / |psi_old,x|^2 and
 *        g = sum_x 2 p_x [Re(E_x - E) d log|psi_x| + Im(E_x - E) d phase_x].
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Spins are int8 values in {-1, +1}, row-major [B][n_sites]; s = 2x - 1 for
 *   the paper's occupation x in {0, 1}.
 * - theta is the flat FP64 parameter vector, gna_num_params() long, laid out as
 *     W_e[2][F], b_e[F], W[nW][2F][F], b[nW][F], v_a[F+2], c_a, v_p[F+2], c_p
 *   with nW = 1 when layers share W, b (tied, Section 2) and nW = L otherwise.
 *   Rows 0..F-1 of W multiply the neighbour message A_hat H, rows F..2F-1 the
 *   node's own row H.  Row 0 of W_e is the embedding of x = 0 (s = -1).
 * - log psi values are FP64 pairs [B][2] = (log|psi|, phase).
 * - Every pointer argument of the compute calls is a DEVICE pointer owned by the
 *   caller.  The library never frees or keeps them past the call.
 * - Every compute call only enqueues work on the context's stream and returns;
 *   none allocates device memory, synchronises, or copies device data to the
 *   host.  Results are valid once the stream has reached them.  The tuning call
 *   gna_autotune is the exception (it synchronises and allocates for its own
 *   duration).
 * - Argument and graph checks are synchronous: on failure the call returns a
 *   nonzero status, enqueues nothing, and gna_last_error() describes why.
 *   A launch failure returns GNA_HIP_ERROR.  Numerical trouble (non-finite
 *   values) is not an error status; gna_isgo_grad reports it in stats[7].
 * - One context must not be used from two host threads at once.
 * - B = 0 is valid for every call: nothing is computed, outputs that are
 *   reductions (grad, stats, n_evals) are still written.
 */
#ifndef GNA_H
#define GNA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gna_ctx gna_ctx;
typedef int32_t gna_status;

enum {
  GNA_OK = 0,
  GNA_INVALID_ARG = 1,   /* bad pointer, size, batch above max_batch, ... */
  GNA_BAD_GRAPH = 2,     /* endpoint out of range, self-loop, repeated bond */
  GNA_UNSUPPORTED = 3,   /* shape outside what the kernels are built for */
  GNA_OUT_OF_MEMORY = 4, /* workspace allocation failed (gna_init, gna_autotune) */
  GNA_HIP_ERROR = 5      /* a HIP runtime call or kernel launch failed */
};

/* Arithmetic of the layer products (Eq. 1).  The readout (the per-node head dot
 * products v . H^L and their sum over sites), the log-psi differences, the local
 * energy sums, the ISGO weights and statistics are FP64 in every mode.
 *   GNA_FP64: everything FP64 (MFMA f64).
 *   GNA_FP32: operands, aggregation and tanh FP32, FP32 MFMA accumulation.
 *   GNA_BF16: weights rounded to bfloat16; each FP32 activation enters the
 *             MFMA as the pair hi + lo of bfloat16 values (two products, about
 *             16 significant bits); aggregation, accumulation and tanh in FP32;
 *             the readout is taken in FP64 from the FP32 last-layer output.
 *             Under GNA_ACT_RELU_LN each weight is a hi + lo pair as well
 *             (three products: hi x hi, hi x lo, lo x hi).
 *   GNA_BF16_1X: as GNA_BF16 but each activation is rounded to the nearest
 *             bfloat16 and each product is a single MFMA (about 8 significant
 *             bits per operand).                                             */
enum { GNA_FP64 = 0, GNA_FP32 = 1, GNA_BF16 = 2, GNA_BF16_1X = 3 };

/* How gna_local_energy and gna_metropolis_sweep evaluate log psi(s^ij):
 *   GNA_ELOC_FULL: every exchanged configuration through all L layers.
 *   GNA_ELOC_INCREMENTAL: only the nodes within graph distance l of the two
 *     exchanged sites are recomputed at layer l (the rest of the configuration
 *     is unchanged there), from per-sample planes of the base configuration kept
 *     in device memory (2 L x N x F values per sample).  The recomputed rows use
 *     the same arithmetic as the full evaluation, so both modes give the same
 *     log psi differences up to the order of the final FP64 sum.  The sampler
 *     keeps each chain's planes current: an accepted proposal's rows stay, a
 *     rejected one is recomputed for the unexchanged configuration.
 *     Needs tied weights and n_layers >= 1.                                   */
enum { GNA_ELOC_FULL = 0, GNA_ELOC_INCREMENTAL = 1 };

/* The nonlinearity f of Eq. 1, applied after every layer and to the embedding:
 *   GNA_ACT_TANH:    f = tanh.
 *   GNA_ACT_RELU_LN: the paper's choice (Section 2): ReLU, then a layer
 *                    normalisation over the F features of each node,
 *                    (y - mean y) / sqrt(var y + 1e-5), biased variance, no
 *                    affine parameters.  The row statistics are reduced in a
 *                    fixed order, so incremental and full evaluations agree.
 *                    Single bfloat16 weights would miss the BF16 bound (the
 *                    normalised layers carry their rounding to the output at
 *                    unit scale: about 0.1 per site at 432 sites, L = 6,
 *                    F = 64), so GNA_BF16 uses split (hi + lo) weights here
 *                    and needs n_features a multiple of 32; gna_init returns
 *                    GNA_UNSUPPORTED for GNA_BF16_1X with this activation, and
 *                    for GNA_BF16 with n_features = 16.                       */
enum { GNA_ACT_TANH = 0, GNA_ACT_RELU_LN = 1 };

typedef struct {
  int32_t n_sites;          /* N >= 2 */
  int32_t n_edges;          /* |E| >= 0 */
  const int32_t *edges;     /* HOST pointer [n_edges][2], copied by gna_init;
                               0 <= i, j < N, i != j, no repeated unordered pair.
                               Periodic boundaries are part of the edge list. */
  int32_t n_features;       /* F: 16, 32 or 64 */
  int32_t n_layers;         /* L: 0 .. 16 applications of Eq. 1 */
  int32_t tied;             /* 1: one W, b shared by all layers (the paper's
                               choice, Section 2); 0: one per layer */
  int32_t precision;        /* GNA_FP64 / GNA_FP32 / GNA_BF16 / GNA_BF16_1X */
  double jz, jxy;           /* Heisenberg couplings; the isotropic model is 1, 1 */
  int32_t max_batch;        /* largest B any call will pass (sizes the workspace) */
  int32_t eloc_mode;        /* GNA_ELOC_FULL or GNA_ELOC_INCREMENTAL (tied weights) */
  int32_t activation;       /* f of Eq. 1: GNA_ACT_TANH or GNA_ACT_RELU_LN */
  int32_t reserved;         /* must be 0 */
  int64_t act_budget_bytes; /* device bytes the reverse pass may use for stored
                               per-layer activations; 0 = library default.  The
                               reverse pass recomputes activations per sample, so
                               this bounds its concurrency, not its result. */
  void *stream;             /* hipStream_t every call enqueues on (NULL = default) */
} gna_config;

/* Validate cfg, copy the graph, build A_hat, and allocate the device workspace.
 * On success *out owns everything; release it with gna_destroy.  On failure
 * *out is NULL and gna_last_error(NULL) describes the problem.              */
gna_status gna_init(const gna_config *cfg, gna_ctx **out);

/* Free the context and its workspace (waits for the context's stream first).
 * NULL is ignored. */
void gna_destroy(gna_ctx *ctx);

/* Length of theta for this context's F, L and weight sharing. */
int64_t gna_num_params(const gna_ctx *ctx);

/* Text of the last error on ctx (or of the last failed gna_init when ctx is
 * NULL).  Valid until the next call on the same context. */
const char *gna_last_error(const gna_ctx *ctx);

/* Change the stream later calls enqueue on. */
gna_status gna_set_stream(gna_ctx *ctx, void *stream);

/* log psi(s) of Eq. 1 plus the two-head readout, for B configurations.
 * theta: [P] FP64; spins: [B][N] int8; logpsi: [B][2] FP64 output.          */
gna_status gna_logpsi(gna_ctx *ctx, const double *theta, const int8_t *spins,
                      int32_t B, double *logpsi);

/* Heisenberg local energy of each configuration (Section 3's E_x), complex:
 * eloc [B][2] FP64 = (Re, Im).  log psi(s) and log psi(s^ij) for every
 * anti-aligned bond are evaluated in-kernel with the same arithmetic, so the
 * differences cancel exactly outside the swapped sites' receptive field.
 * n_evals (device int64, may be NULL) receives B + sum_x #anti-aligned bonds,
 * the number of log-psi evaluations performed.                            */
gna_status gna_local_energy(gna_ctx *ctx, const double *theta, const int8_t *spins,
                            int32_t B, double *eloc, int64_t *n_evals);

/* gna_local_energy for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and results, with the call's scratch (base log psi, per-work-item
 * partial sums and counts, the pipelined kernel's exchange terms, and the
 * evaluation counter when n_evals is NULL) in a static device array of the
 * library, 64 MiB on each GPU it runs on, held until the process ends, instead
 * of the context's workspace.  The call performs no allocation of any kind; the
 * context's persistent buffers (weight fragments, and in GNA_ELOC_INCREMENTAL
 * mode the base planes) come from gna_init.  Arguments as gna_local_energy.
 * GNA_INVALID_ARG, with nothing enqueued, when B needs more scratch than the
 * array holds (about B * (16 + 36 * bond chunks) bytes, plus B * 16 * n_edges
 * with the layer-pipelined local-energy kernel; 2048 samples of the 432-site
 * Kagome workload need about 29 MiB).
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (two streams, two host threads, two contexts) race and must be
 * serialised by the caller.  GNA_HIP_ERROR if the array's address could not be
 * obtained at gna_init.                                                      */
gna_status gna_local_energy_noalloc(gna_ctx *ctx, const double *theta, const int8_t *spins,
                                    int32_t B, double *eloc, int64_t *n_evals);

/* n_sweeps * N Metropolis proposals per chain (one chain per row; Section 3's
 * Markov chain for |psi|^2).  Proposal k of chain b draws one Philox4x32-10
 * block with counter (low32(t), high32(t), b, 0), t = counter_base + k, and key
 * (low32(seed), high32(seed)); word 0 picks bond (w0 * n_edges) >> 32, word 1
 * gives u = (w1 + 0.5) 2^-32.  An aligned bond is an identity step; otherwise
 * the swap is accepted iff u < exp(2 Re[log psi(s^ij) - log psi(s)]).
 * spins [B][N] and logpsi [B][2] are read and updated in place; logpsi must
 * hold the chains' current values (e.g. from gna_logpsi on this context).
 * In GNA_ELOC_INCREMENTAL mode the difference is taken from the recomputed
 * receptive field, and logpsi is overwritten at the end with log psi of the
 * final configurations, summed from the per-node readout terms the sampler
 * keeps current, in the full evaluation's order (bitwise what gna_logpsi
 * returns for them).
 * n_accept: [B] int32 output (accepted swaps), may be NULL.                */
gna_status gna_metropolis_sweep(gna_ctx *ctx, const double *theta, int8_t *spins,
                                double *logpsi, int32_t B, int32_t n_sweeps,
                                uint64_t seed, uint64_t counter_base, int32_t *n_accept);

/* One variational step on device-resident state, everything enqueued on the
 * context's stream with no host synchronisation, so that a caller can capture it
 * in a HIP graph and replay it (Section 3's loop of sampling, energy and update):
 *   1. logpsi <- log psi(spins)                               (gna_logpsi)
 *   2. n_sweeps Metropolis sweeps with counter base *counter  (gna_metropolis_sweep)
 *   3. *counter += n_sweeps * N                               (device side)
 *   4. ISGO gradient with logpsi as the sampling distribution (gna_isgo_grad;
 *      grad [P], stats [8], eloc [B][2] or NULL)
 *   5. theta -= lr * grad                                     (gna_sgd_update)
 * counter: device uint64, read and advanced on the device, so every replay of a
 * captured step draws new proposals.  All pointers are device pointers.      */
gna_status gna_step(gna_ctx *ctx, double *theta, int8_t *spins, double *logpsi, int32_t B,
                    int32_t n_sweeps, uint64_t seed, uint64_t *counter, double lr, double *grad,
                    double *stats, double *eloc, int32_t *n_accept);

/* The bond Hamiltonian of gna_local_energy (and so of gna_isgo_grad, gna_step):
 *   E(s) = sum_<ij> [ jz s_i s_j / 4 + hb (s_i + s_j) / 4 + cb
 *                     + (jxy / 2) [s_i != s_j] psi(s^ij) / psi(s) ]
 * gna_init sets (jz, jxy) from the config and hb = cb = 0 (the Heisenberg model of
 * Section 3).  The hard-core bosons of Eq. 4 (hopping t, interaction V, occupation
 * n = (1 + s)/2) are jz = V, jxy = -2t, hb = V, cb = V/4.  Host-side, synchronous;
 * applies to every later call.  INVALID_ARG for a non-finite value.          */
gna_status gna_set_couplings(gna_ctx *ctx, double jz, double jxy, double hb, double cb);

/* Tile and workgroup shapes of the incremental kernels chosen by measurement:
 * times gna_local_energy on (theta, spins[B]) for the candidate shapes (jobs in
 * flight per workgroup, 8 or 16 waves, one or two samples in flight per XCD, and
 * the layer-pipelined kernels, jobs_in_flight 0, with 8 or 16 waves),
 * then one Metropolis sweep of a copy of the batch (spins is not modified) for
 * the same candidates; each kernel keeps its fastest shape, for this context and
 * for every later context of the same signature (N, n_edges, degree histogram,
 * F, L, precision) in this process.  Unlike the compute calls it synchronises
 * the context's stream and allocates a temporary copy of the batch (B*N bytes
 * plus 12*B) for the call: call it after gna_init, outside any graph capture.
 * chosen [8] (host, may be NULL): local energy jobs in flight (0: pipelined),
 * waves, samples per XCD, microseconds per call; sweep jobs in flight, waves, tiles per wave,
 * microseconds per one-sweep call.  In GNA_ELOC_FULL mode there is nothing to
 * tune: returns GNA_OK, chosen zeros.  OUT_OF_MEMORY if the copy cannot be had.  */
gna_status gna_autotune(gna_ctx *ctx, const double *theta, const int8_t *spins, int32_t B,
                        int32_t *chosen);

/* Pin the shape of the incremental kernels instead of measuring it (a shape
 * reported by gna_autotune or gna_config_info earlier, or one to profile).
 * which: 1 the local-energy kernel, 2 the sweep kernel, 3 both.  jobs_in_flight
 * in [1, 8]: exchanged configurations per workgroup advanced layer by layer
 * together; waves 16 selects the one-tile-per-wave variant (1024-thread bound: it
 * launches one wave per tile, at most 16), 1..8 the variant with up to four tiles
 * per wave, capped at the jobs' tile count (16-node tiles of the largest L-hop
 * ball).  jobs_in_flight 0: the layer-pipelined kernels, L + 2 jobs per
 * workgroup at staggered layers, each pair of barriers advancing every job by one
 * layer; waves 8 or 16, one of them preparing the jobs; tanh with FP32 or BF16
 * only, and only where the jobs' tiles fit in the waves' registers and their rows
 * in LDS.  samples_per_xcd in
 * [1, 8] (local energy only).  gna_autotune and gna_config_info report waves
 * the same way, so a reported shape can be pinned again.
 * Results do not depend on the shape beyond the order of the final FP64 sums.
 * INVALID_ARG outside those ranges or in GNA_ELOC_FULL mode; UNSUPPORTED when the
 * shape does not fit in LDS or needs more than four tiles per wave (pipelined:
 * more tiles than the waves' registers hold, FP64, or ReLU + layer
 * normalisation); on error the previous shapes stay.  Host-side; applies to
 * every later call.                                                          */
gna_status gna_set_shape(gna_ctx *ctx, int32_t which, int32_t jobs_in_flight, int32_t waves,
                         int32_t samples_per_xcd);

/* Shape in use (host array, n entries at most 11): eloc_mode, jobs in flight (0: pipelined),
 * waves per workgroup, tiles per wave, samples per XCD, precision, F, L, then the
 * sweep kernel's jobs in flight, waves and tiles per wave (in GNA_ELOC_FULL mode
 * the full evaluator's waves and tiles per wave).  Returns 11, or -1 for a NULL
 * context.                                                                   */
int32_t gna_config_info(const gna_ctx *ctx, int32_t *info, int32_t n);

/* Reverse pass of Eq. 1 and the readout, the vector-Jacobian product from
 * which Eq. 2 and Eq. 3 form the energy gradient (Section 3):
 *   grad[P] = sum_x cot[x][0] d log|psi(s_x)|/dtheta
 *           + cot[x][1] d phase(s_x)/dtheta   (overwritten).
 * The forward pass is recomputed per sample and its per-layer activations are
 * held for the reverse pass (FP64 in GNA_FP64, FP32 in the other modes), at most
 * act_budget_bytes of them at once: a larger batch is processed in chunks, whose
 * per-parameter sums are accumulated in FP64.  cot: [B][2].                 */
gna_status gna_logpsi_vjp(gna_ctx *ctx, const double *theta, const int8_t *spins,
                          int32_t B, const double *cot, double *grad);

/* One ISGO update's gradient (Eq. 3) for samples drawn under an earlier theta:
 * new log psi, local energies under the new psi, self-normalised weights
 *   r_x = n_x exp(2 Re(lp_new - lp_old) - m),  m = max_x 2 Re(lp_new - lp_old),
 *   p_x = r_x / sum r,  E = sum p_x E_x,
 * then grad = reverse pass with cotangents 2 p_x (Re(E_x - E), Im(E_x - E)).
 * logpsi_old: [B][2]; counts: [B] FP64 multiplicities or NULL (all 1);
 * grad: [P] output; stats: [8] output = {Re E, Im E, sum p|E_x - E|^2,
 *   ESS = (sum r)^2 / sum r^2, sum r, m, n_evals, nonfinite flag (0/1)};
 * eloc: [B][2] output or NULL.                                             */
gna_status gna_isgo_grad(gna_ctx *ctx, const double *theta, const int8_t *spins,
                         const double *logpsi_old, const double *counts, int32_t B,
                         double *grad, double *stats, double *eloc);

/* Section 3's grouping of duplicated sampled states into unique states with
 * counts, on the device: uniq[0..U) are the distinct rows of spins in the order
 * of their first occurrence, counts[g] how many rows equal uniq[g] (FP64, ready
 * for the counts argument of gna_isgo_grad), and *n_unique = U.  Rows
 * uniq[U..B) repeat uniq[0] with count 0, so the whole [B] output may be passed
 * on unchanged; passing B' = U rows (after reading n_unique) skips them.
 * spins: [B][N] int8 (device); uniq: [B][N] int8 (device, must not overlap
 * spins); counts: [B] FP64 (device); n_unique: one int32 (device).  Rows are
 * matched by a 64-bit hash of their packed spins and then compared in full, so
 * distinct rows never share a group; equal rows always do unless their hash
 * collides with another row's (probability about B^2 / 2^65), in which case a
 * group can appear twice with its count split, which leaves every count-weighted
 * sum unchanged.  Asynchronous, no allocation, graph-capturable.              */
gna_status gna_group_duplicates(gna_ctx *ctx, const int8_t *spins, int32_t B, int8_t *uniq,
                                double *counts, int32_t *n_unique);

/* Section 3's update theta <- theta - alpha * grad, in place on the device. */
gna_status gna_sgd_update(gna_ctx *ctx, double *theta, const double *grad, double alpha);

/* Kernel timing for benchmarks: while enabled, every kernel the context launches
 * is bracketed by two HIP events recorded on the context's stream.
 * gna_profile_read waits for the stream, then returns, per kernel name, the
 * number of launches and their summed duration in milliseconds since the last
 * read (max_entries rows of names[64 chars], launches, total_ms); the return value
 * is the number of distinct kernels, or -1 on error.  Reading clears the record. */
gna_status gna_profile_enable(gna_ctx *ctx, int32_t on);
int32_t gna_profile_read(gna_ctx *ctx, int32_t max_entries, char *names,
                         int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* GNA_H */
