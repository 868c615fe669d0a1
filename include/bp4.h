/*
 * bp4.h -- C ABI of the MI355X (gfx950) flooding-schedule GF(4) belief
 * propagation library: traditional LLR-BP4 and the Momentum-BP, AdaGrad-BP
 * and EWAInit-BP variants of Chen, Yi, Liang, Wang, "Improved Belief
 * Propagation Decoding Algorithms for Surface Codes" (arXiv 2407.11523), on
 * very large batches of syndromes.
 *
 * Conventions (all entry points)
 *   - Pauli code per qubit, one byte: bit0 = x, bit1 = z (I=0, X=1, Z=2, Y=3).
 *   - Per-qubit LLR triples are (X, Y, Z), the order of section II-B1.
 *   - Syndrome bits are bytes in {0, 1}; the check sign is (-1)^{s_c}
 *     (eq. h_update).
 *   - "dev" pointers are device memory of the current HIP device, "host"
 *     pointers host memory.  The library allocates no device memory: the
 *     caller passes every device buffer (graph image, workspace, outputs).
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Device work is enqueued on it asynchronously; host arguments are read
 *     before the call returns.
 *   - Every function returns BP4_OK (0) or a negative error code; the
 *     message of the calling thread's last error is bp4_last_error().
 *     Arguments are validated on the host before anything is launched; on
 *     error nothing is enqueued.
 */
#ifndef BP4_H
#define BP4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BP4_OK = 0,
    BP4_EINVAL = -1,       /* bad shape, pointer, entry or parameter */
    BP4_ENONCOMM = -2,     /* two stabilizer rows anticommute */
    BP4_EDEGREE = -3,      /* a check or qubit degree exceeds the compiled maximum */
    BP4_EWORKSPACE = -4,   /* workspace or graph buffer too small */
    BP4_EHIP = -5,         /* a HIP runtime call failed */
    BP4_EUNSUPPORTED = -6  /* size beyond what the kernels index */
};

/* Decoder variants (section III). */
typedef enum {
    BP4_BP = 0,        /* traditional LLR-BP4, section II-B1 */
    BP4_MOMENTUM = 1,  /* Momentum-BP, parallel form, eqs. mombp1-mombp3 */
    BP4_ADAGRAD = 2,   /* AdaGrad-BP, eq. boost */
    BP4_EWAINIT = 3,   /* EWAInit-BP, eq. EWAInit, Algorithm 2 */
    BP4_AEWA = 4       /* AEWA-BP (appendix on adaptive MBP): EWAInit-BP restarted with the
                          next discount of a list until the syndrome is met */
} bp4_variant;

/* Hyperparameters of one decode.
 *   alpha: Momentum step (learning rate), AdaGrad boost learning rate,
 *          EWAInit discount factor.  Momentum / EWAInit need 0 <= alpha <= 1,
 *          AdaGrad alpha > 0.  Ignored by BP.
 *   gamma: Momentum decay, 0 <= gamma < 1.
 *   eps:   AdaGrad epsilon, > 0.
 *   llr_clamp: every message is clamped to [-llr_clamp, llr_clamp], > 0.
 *   max_iter: iter_max >= 1.
 *   stop_on_syndrome: 1 halts a shot at the first iteration whose hard
 *          decision reproduces its syndrome (Algorithm 2); 0 runs max_iter.
 *   adagrad_g_from_t1: 1 also accumulates the squared gradient at t = 1.
 *   alpha_last, alpha_steps (AEWA only): attempt k = 0 .. alpha_steps - 1 is a
 *          fresh EWAInit decode of up to max_iter iterations with discount
 *          alpha + (alpha_last - alpha) * k / (alpha_steps - 1) (alpha for a
 *          single step); the first attempt that meets the syndrome is the
 *          result, else the last one.  Both discounts in [0, 1], 1 <=
 *          alpha_steps <= 64, stop_on_syndrome must be 1; `iters` reports the
 *          iterations of all attempts.  Ignored by the other variants.
 *   serial: 0 flooding schedule (all checks, then all qubits; Algorithm 2);
 *          1 serial schedule (Algorithm 1: qubit by qubit in index order, each
 *          qubit's incoming check messages from the current messages of the
 *          check's other qubits, then its posterior and outgoing messages).
 *          On the LDS kernel (the automatic choice when 64-lane groups fit)
 *          the sweep runs level by level: a qubit's level is one more than the
 *          highest level of an earlier qubit sharing a check with it, so the
 *          qubits of a level are updated together with the sequential result;
 *          wave groups of group_lanes 1, 2, 4, ..., 64 lanes per shot
 *          (block_shots must be 0).  Large codes take the single-pass HBM
 *          kernel: one lane per shot, the same level sweep with each shot's
 *          messages updated in place in HBM and a workgroup barrier per level
 *          (also available for small codes with BP4_KERNEL_GATHER); the SOA
 *          kernel runs it one lane per shot, qubit by qubit.  All give the same
 *          bits.  bp4_decode_mixed and
 *          bp4_decode_plain answer EUNSUPPORTED. */
typedef struct {
    int32_t variant;
    int32_t max_iter;
    int32_t stop_on_syndrome;
    int32_t adagrad_g_from_t1;
    float alpha;
    float gamma;
    float eps;
    float llr_clamp;
    float alpha_last;
    int32_t alpha_steps;
    int32_t serial;
} bp4_params;

/* Opaque host object describing one code's Tanner graph (section II-B1). */
typedef struct bp4_graph bp4_graph;

#define BP4_ALLOW_ANTICOMMUTING 1u   /* graph_create flag: skip the commutation check */

/* Build the Tanner graph of the symplectic check matrix (hx | hz), host
 * uint8 arrays [m][n] row-major; row i is the stabilizer S_i, entry j its
 * Pauli on qubit j (section II-B1).  Edge (i, j) exists where the entry is
 * not I; its label is the GF(4) entry H_ij.  The inputs are copied.
 * A graph whose checks and qubits all have degree <= 4 is narrow and runs on
 * every kernel; otherwise it is wide (checks of degree <= 8, qubits <= 7, as
 * the bivariate bicycle and 3D Chamon codes of section IV-C need) and runs on
 * the LDS kernel (flooding and serial schedules), the plain decoder, the sampler
 * and bookkeeping (the HBM kernels and the unrolled path answer EUNSUPPORTED;
 * bp4_decode_mixed runs a batch of wide and narrow codes as two persistent
 * launches in stream order, one per build).
 * Errors: EINVAL (m, n <= 0, entries not 0/1, empty row or column, NULL),
 * ENONCOMM (rows anticommute, unless BP4_ALLOW_ANTICOMMUTING), EDEGREE
 * (check degree above 8 or qubit degree above 7), EUNSUPPORTED (n > 16383 or
 * more than 65534 edges). */
int bp4_graph_create(const uint8_t *hx, const uint8_t *hz, int32_t m, int32_t n,
                     uint32_t flags, bp4_graph **out);

/* Attach a logical-operator basis (host uint8 [nlog][n] each, the x and z
 * parts) used by bp4_bookkeep to tell undetected logical errors from
 * success (section IV).  Errors: EINVAL. */
int bp4_graph_set_logicals(bp4_graph *g, const uint8_t *lx, const uint8_t *lz, int32_t nlog);

/* Optional locality hint of a narrow graph: xy, host int32 [n][2], a position
 * of each qubit on a 2-D layout of the code (any integer units, e.g. lattice
 * coordinates).  Only the order in which the single-pass HBM kernel walks the
 * qubits depends on it: strips of the layout walked row by row join the
 * candidate orders, and the one with the fewest misses in a model of the
 * kernel's L2 reuse is kept, which decides how many of its message re-reads L2
 * serves.  Decoding results never depend on it.  The input is copied; call
 * bp4_graph_upload afterwards (an uploaded image keeps the previous order).
 * Errors: EINVAL (NULL), EUNSUPPORTED (wide graph: no single-pass kernel). */
int bp4_graph_set_coords(bp4_graph *g, const int32_t *xy);

/* Sizes of the graph: qubits, checks, edges, maximum check and qubit degree. */
int bp4_graph_info(const bp4_graph *g, int32_t *n, int32_t *m, int32_t *nnz,
                   int32_t *max_cdeg, int32_t *max_vdeg);

/* Bytes of device memory that bp4_graph_upload fills. */
int bp4_graph_device_bytes(const bp4_graph *g, size_t *bytes);

/* Copy the graph image (edge lists, labels, logicals) into dev_buf
 * (caller-owned, >= bp4_graph_device_bytes, 256-byte aligned).  Blocks until
 * the copy is done.  Call again after bp4_graph_set_logicals and
 * bp4_graph_set_coords.
 * Errors: EINVAL, EWORKSPACE (buffer too small), EHIP. */
int bp4_graph_upload(const bp4_graph *g, void *dev_buf, size_t bytes, void *stream);

void bp4_graph_destroy(bp4_graph *g);

/* Canonical edge order: the nonzeros of H in row-major order.  Writes, for
 * each canonical edge k, its check and qubit (host int32 [nnz] each). */
int bp4_graph_edges(const bp4_graph *g, int32_t *check, int32_t *qubit);

/* Device workspace bytes bp4_decode needs for `shots` shots with the automatic
 * kernel choice (a queue counter for the LDS kernel; the column records of the
 * single-pass HBM kernel; the SOA kernel's lane-resident message and state
 * arrays only with its tuning fields). */
int bp4_workspace_bytes(const bp4_graph *g, const bp4_params *p, int64_t shots, size_t *bytes);

/* Sample i.i.d. Pauli errors and their syndromes (section IV: each qubit is
 * X, Y, Z with probabilities pX, pY, pZ).  Shot i (global index shot0 + i)
 * uses Philox4x64-10 (Salmon et al., SC'11) with key (seed, stream_id) and
 * counter (shot0 + i, q / 8, 0, 0); qubit q takes 32-bit half (q % 2) of
 * output word (q % 8) / 2 and compares it with the integer thresholds
 * thr = (tX, tY, tZ) of 2^32: u < tX -> X, < tX+tY -> Y, < tX+tY+tZ -> Z.
 * Writes err dev [shots][n] and synd dev [shots][m], s_c = sum_v <H_cv, E_v>
 * mod 2.  Errors: EINVAL (thresholds sum >= 2^32, NULL), EHIP. */
int bp4_sample(const bp4_graph *g, const void *dev_graph, int64_t shots, int64_t shot0,
               const uint32_t thr[3], uint64_t seed, uint64_t stream_id,
               uint8_t *err, uint8_t *synd, void *stream);

/* Prior LLRs of the decoder input (section II-B1): for each qubit v with
 * error probabilities probs dev double [n][3] = (p_X, p_Y, p_Z),
 *     prior dev float [n][3]:  Pi_{v,W} = ln(p_v^I / p_v^W),  p_v^I = 1 - p_X - p_Y - p_Z,
 * evaluated in double precision and rounded to float.  (The paper prints
 * ln((1 - p)/p) for the probability vector; lambda is a commutation LLR only
 * if e^{-Pi_W} = p_W / p_I, which fixes this reading.)  The probabilities are
 * device data, so the host cannot check them: an entry with p_W <= 0,
 * p_I <= 0 or a non-finite probability gets a NaN prior, and a decode from
 * NaN priors reports its shots as not converged.  The Python binding checks
 * the probabilities before the call.  Errors: EINVAL (n outside [1, 16383],
 * NULL), EHIP. */
int bp4_prior_llr(int32_t n, const double *probs, float *prior, void *stream);

/* Decode `shots` syndromes (synd dev [shots][m]) with prior LLRs
 * prior_llr dev [n][3], Pi_{v,W} = ln(p_v^I / p_v^W) (section II-B1,
 * Algorithm 2 input), by flooding-schedule BP of the chosen variant.  Per
 * shot: est dev [shots][n] (hard decision, section II-B1), conv dev [shots]
 * (1 iff the hard decision reproduces the syndrome at the last iteration
 * run), iters dev [shots] (iterations run, 1..max_iter).  ws is a device
 * workspace of >= bp4_workspace_bytes.
 * Errors: EINVAL (parameters out of range, NULL), EWORKSPACE, EHIP. */
int bp4_decode(const bp4_graph *g, const void *dev_graph, const bp4_params *p, int64_t shots,
               const float *prior_llr, const uint8_t *synd,
               uint8_t *est, uint8_t *conv, int32_t *iters,
               void *ws, size_t ws_bytes, void *stream);

/* Launch choices of the decode kernels.  kernel: BP4_KERNEL_AUTO, _LDS, _SOA
 * or _GATHER (below).  Lane mapping of the LDS kernel (0 and 0: picked by lane use
 * and occupancy): group_lanes 4, 8, 16, 32 or 64 = that many lanes of one
 * wavefront decode one shot (lane r owns checks and qubits r, r + G, ...);
 * block_shots S in [1, 512] (with group_lanes 0 or 512) = S shots share the
 * 512 lanes of a workgroup, which walk the S*m check and S*n qubit items of
 * the S shots in passes of 512 (at most 64 check items per lane);
 * group_lanes 128, 256 and 512 alone mean block_shots 4, 2 and 1.  Results do
 * not depend on the mapping.
 * lds_bytes: if larger than the code's own layout, each workgroup of the LDS
 * kernel reserves this much LDS (so a single-code launch runs at the
 * occupancy of a mixed launch that needs it; 0: the layout's size).
 * soa_lanes: shots the SOA kernel keeps in flight (0: 262,144; rounded up to
 * a multiple of 256 and capped by the shot count); the SOA workspace grows
 * with it.  soa_iter_block: iterations per SOA launch, after which the shots
 * still running are packed onto fully populated wavefronts (0: 24); results
 * do not depend on it.  gather_waves: wavefronts per workgroup of the
 * single-pass HBM kernel, 4, 8 or 16 (0: 16; 64 shots per workgroup, 32
 * wavefronts per CU); results do not depend on it.  group_lanes, block_shots
 * and lds_bytes select the LDS kernel under AUTO, soa_lanes and
 * soa_iter_block the SOA kernel, gather_waves the single-pass HBM kernel;
 * each group is rejected with the other kernels.  reserved: 0. */
typedef struct {
    int32_t group_lanes;
    int32_t lds_bytes;
    int32_t kernel;
    int32_t soa_lanes;
    int32_t soa_iter_block;
    int32_t block_shots;
    int32_t gather_waves;
    int32_t reserved;
} bp4_tuning;

/* Decode kernels.  LDS: a lane group per shot, state in LDS (small and medium
 * codes).  SOA: one lane per shot, messages and state in HBM as
 * structure-of-arrays [slot][lane], a check pass and a qubit pass per
 * iteration, the shots still running packed between launches (large codes;
 * every variant, both schedules, the verification outputs).  GATHER: one
 * lane per shot, 64 shots per workgroup, one pass over HBM per iteration:
 * each qubit reads its checks' other messages (L2 serves the re-reads of the
 * neighbouring qubits) and writes its own; the syndrome test runs inside the
 * pass and a finished shot's lane takes the next shot at once (large codes;
 * every variant, AEWA's unsolved shot keeping its lane for the next attempt,
 * and both schedules, the serial one as a level sweep with the messages
 * updated in place; at most 4,079 checks, no verification outputs).
 * AUTO: LDS unless even one shot per workgroup would need more than 80 KB of
 * LDS; then GATHER where it applies, else SOA. */
enum { BP4_KERNEL_AUTO = 0, BP4_KERNEL_LDS = 1, BP4_KERNEL_SOA = 2, BP4_KERNEL_GATHER = 3 };

/* Device workspace bytes of the SOA kernel for `shots` shots with soa_lanes
 * lanes in flight (0: the default): per lane, two records (the running one
 * and the packed one of the next launch) of every message, the posterior
 * (all variants but BP), the momentum or AdaGrad accumulator and the
 * syndrome bits, plus the decisions.  Errors: EINVAL (negative shots or
 * lanes). */
int bp4_soa_workspace_bytes(const bp4_graph *g, const bp4_params *p, int64_t shots, int32_t soa_lanes,
                            size_t *bytes);

/* Device workspace bytes of the single-pass HBM kernel (flooding decode of
 * section II-B1 for large codes) for `shots` shots and gather_waves
 * wavefronts per workgroup (0: 16): the shot queue head, the initial-message
 * table (4 words per check) and, for each of the
 * min(ceil(shots / 64), 256 x 32 / gather_waves) workgroups in flight, two
 * records of 64 columns holding 4 message words per check and 3 posterior
 * words (6 with the Momentum or AdaGrad accumulator) per qubit.
 * Errors: EINVAL (NULL, negative shots, gather_waves not 0, 4, 8 or 16,
 * parameters out of range). */
int bp4_gather_workspace_bytes(const bp4_graph *g, const bp4_params *p, int64_t shots, int32_t gather_waves,
                               size_t *bytes);

/* As bp4_decode, with launch choices `tune` (NULL: automatic; with
 * tune->kernel = BP4_KERNEL_SOA the workspace must hold
 * bp4_soa_workspace_bytes, with BP4_KERNEL_GATHER
 * bp4_gather_workspace_bytes; under AUTO a large code that asks for the
 * verification outputs runs the SOA kernel and needs its workspace) and, for
 * verification, the state after the last iteration run: q_out dev
 * [shots][n][3] posterior LLRs Q; mvc_out and mcv_out dev [shots][nnz]
 * variable-to-check and check-to-variable messages in canonical edge order.
 * Each of q_out and the (mvc_out, mcv_out) pair may be NULL; writing them
 * slows the decode.  Errors: as bp4_decode; EINVAL for a group size the code
 * does not fit (more than 64 checks per lane, or LDS exhausted). */
int bp4_decode_ex(const bp4_graph *g, const void *dev_graph, const bp4_params *p,
                  const bp4_tuning *tune, int64_t shots, const float *prior_llr,
                  const uint8_t *synd, uint8_t *est, uint8_t *conv, int32_t *iters,
                  float *q_out, float *mvc_out, float *mcv_out,
                  void *ws, size_t ws_bytes, void *stream);

/* LDS bytes per workgroup the LDS decode kernel needs for this code, variant
 * and lane mapping (group_lanes, block_shots as in bp4_tuning; not both 0).
 * Errors: EINVAL if the mapping is invalid or leaves more than 64 checks per
 * lane. */
int bp4_lds_layout_bytes(const bp4_graph *g, const bp4_params *p, int32_t group_lanes, int32_t block_shots,
                         size_t *bytes);

/* One code of a mixed batch: its graph, parameters, shots and buffers (as the
 * arguments of bp4_decode).  group_lanes and block_shots as in bp4_tuning
 * (both 0: automatic). */
typedef struct {
    const bp4_graph *graph;
    const void *dev_graph;
    bp4_params params;
    int64_t shots;
    const float *prior_llr;
    const uint8_t *synd;
    uint8_t *est;
    uint8_t *conv;
    int32_t *iters;
    int32_t group_lanes;
    int32_t block_shots;
} bp4_code_batch;

#define BP4_MAX_MIXED_CODES 16

/* Device workspace bytes of bp4_decode_mixed (one shot queue per code). */
int bp4_mixed_workspace_bytes(int32_t ncodes, size_t *bytes);

/* Decode the syndromes of up to BP4_MAX_MIXED_CODES codes (different sizes,
 * families, variants, parameters and shot counts) in one persistent launch:
 * each workgroup stages one code's graph in LDS and its lane groups pull that
 * code's shots from a queue, then the workgroup moves on to the next code
 * (largest first).  Results per code as bp4_decode; bit-identical to decoding
 * each code alone with the same lane mapping.  Errors: as bp4_decode, EINVAL
 * for ncodes outside [1, BP4_MAX_MIXED_CODES]. */
int bp4_decode_mixed(int32_t ncodes, const bp4_code_batch *codes, void *ws, size_t ws_bytes,
                     void *stream);

/* bp4_decode_mixed for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the same
 * launch, inputs, outputs and results, but its scratch memory, the per-code
 * shot-queue heads, is a 256-byte array inside the library's code object (one per
 * GPU, held until the process ends) instead of a caller workspace, and the call
 * allocates nothing.  The heads are cleared by a fill kernel on `stream` before each
 * launch.  Every call on one GPU shares that array: calls that overlap on one GPU
 * (different streams, or threads) race and must not be issued.  Errors: as
 * bp4_decode_mixed; EINVAL for ncodes outside [1, BP4_MAX_MIXED_CODES] (the
 * array's limit), EHIP if the array's device address cannot be obtained. */
int bp4_decode_mixed_noalloc(int32_t ncodes, const bp4_code_batch *codes, void *stream);

/* Device workspace bytes of bp4_decode_plain: messages, per-qubit state and
 * hard decisions of every shot in HBM. */
int bp4_plain_workspace_bytes(const bp4_graph *g, const bp4_params *p, int64_t shots, size_t *bytes);

/* The textbook GPU mapping of the same decoder, the reference point of the
 * persistent kernels: one kernel per phase per iteration, one thread per
 * (shot, check) or (shot, qubit), messages in HBM, finished shots masked.
 * The host reads the number of unfinished shots after each iteration, so the
 * call blocks until the decode is done; *iterations_run (host, may be NULL)
 * receives the iterations launched.  Same arithmetic per node as bp4_decode,
 * so the outputs are bit-identical.  Errors: as bp4_decode. */
int bp4_decode_plain(const bp4_graph *g, const void *dev_graph, const bp4_params *p, int64_t shots,
                     const float *prior_llr, const uint8_t *synd,
                     uint8_t *est, uint8_t *conv, int32_t *iters,
                     void *ws, size_t ws_bytes, void *stream, int32_t *iterations_run);

/* Classify each shot (section IV): with R = E^ E, fail dev [shots] = 1
 * ("detected": R anticommutes with a stabilizer), 2 ("undetected": R
 * commutes with every stabilizer but not with a logical operator of the
 * basis set by bp4_graph_set_logicals) or 0 (success).  counts dev int64[3]
 * is incremented by the number of shots of each class (the caller zeroes it
 * first).  err, est: dev [shots][n].  Errors: EINVAL (no logicals), EHIP. */
int bp4_bookkeep(const bp4_graph *g, const void *dev_graph, int64_t shots,
                 const uint8_t *err, const uint8_t *est, uint8_t *fail, int64_t *counts,
                 void *stream);

/* ---- Differentiable unrolled BP -----------------------------------------
 * A variant of section III run for exactly T iterations (Algorithm 2 without
 * the early stop) with learnable per-iteration parameters param_t dev float
 * [T][k] and learnable priors Pi^{(0)} dev float [n][3]; messages clamped to
 * [-llr_clamp, llr_clamp] as in bp4_decode.  Built for two variants:
 *   BP4_EWAINIT, k = 1: param_t[t-1] is the discount alpha_t of iteration t
 *   (Pi^{(1)} = Pi^{(0)}, Pi^{(t)} = alpha_t Pi^{(0)} + (1 - alpha_t) Q^{(t-1)},
 *   eq. EWAInit; entry 0 is unused);
 *   BP4_MOMENTUM, k = 2: param_t[t-1] = (alpha_t, gamma_t), the step and decay
 *   of iteration t (g^{(t)} = gamma_t g^{(t-1)} + (1 - gamma_t)(Q^{(t-1)} -
 *   Pi^{(0)} - M^{(t)}), Q^{(t)} = Q^{(t-1)} - alpha_t g^{(t)}, g^{(0)} = 0, eqs.
 *   mombp1-3; the state also keeps g and M, 9 words per qubit instead of 3).
 * Every other variant answers EUNSUPPORTED.
 * Loss: the mean over shots and qubits of
 * ln(1 + sum_W e^{-Q_W^{(T)}}) + Q_{e_v}^{(T)} (Q_I = 0), the negative log of
 * the GF(4) marginal of the sampled error e_v.  The adjoint returns its
 * gradient with respect to param_t and Pi^{(0)}.  The forward keeps the state
 * (messages and posteriors) every ckpt_every iterations in `saved`; the
 * backward recomputes each segment from its checkpoint.
 *
 * Device buffers (caller-allocated): param_t, prior, synd uint8 [shots][m],
 * err uint8 [shots][n] (Pauli codes), saved and ws of the sizes below.
 * Errors: EINVAL (T < 1, ckpt_every < 1, shots < 1, llr_clamp not > 0, NULL
 * pointers, variant outside bp4_variant), EUNSUPPORTED (a variant other than
 * EWAInit or Momentum, a wide graph), EWORKSPACE (saved or ws too small), EHIP. */

/* Bytes of the checkpoint buffer and of the workspace for these sizes. */
int bp4_unrolled_sizes(const bp4_graph *g, int32_t variant, int32_t T, int32_t ckpt_every, int64_t shots,
                       size_t *saved_bytes, size_t *ws_bytes);

/* Forward: writes loss dev double [1] and, if q_out is not NULL, the final
 * posteriors Q^{(T)} dev float [shots][n][3]; fills `saved`. */
int bp4_unrolled_forward(const bp4_graph *g, const void *dev_graph, int32_t variant, int32_t T, int32_t ckpt_every,
                         float llr_clamp, int64_t shots, const float *param_t, const float *prior,
                         const uint8_t *synd, const uint8_t *err, double *loss, float *q_out,
                         void *saved, size_t saved_bytes, void *ws, size_t ws_bytes, void *stream);

/* Backward: with `saved` from the forward of the same inputs, writes
 * dparam_t dev double [T][k] = dloss * dL/dparam_t (EWAInit: entry 0 is 0) and
 * dprior dev double [n][3] = dloss * dL/dPi^{(0)}; dloss is a dev float
 * scalar (NULL: 1). */
int bp4_unrolled_backward(const bp4_graph *g, const void *dev_graph, int32_t variant, int32_t T, int32_t ckpt_every,
                          float llr_clamp, int64_t shots, const float *param_t, const float *prior,
                          const uint8_t *synd, const uint8_t *err, const float *dloss,
                          const void *saved, size_t saved_bytes, double *dparam_t, double *dprior,
                          void *ws, size_t ws_bytes, void *stream);

/* Message of the calling thread's last non-OK return. */
const char *bp4_last_error(void);

/* Library version string. */
const char *bp4_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BP4_H */
