/*
 * libsagms -- batched min-sum decoding of generalized-bicycle QLDPC codes
 * on MI355X (gfx950).  C ABI.
 *
 * Implements the decoding path of Cordova et al., "Syndrome Adaptive Gain
 * Control for Min-Sum Decoding of Quantum LDPC Codes" (arXiv 2605.10433):
 * depolarizing-noise Monte Carlo frames (Section II), their syndromes, and
 * the MS, SMS and SAGMS decoders of Sections II-III (Algorithm 1), with the
 * BP decoder of eq. (bp4_cn) as a comparison.  Decoding is binary: the X
 * part of each error is decoded on the Tanner graph of one CSS check matrix
 * (H_Z for GB codes) from its syndrome, with a per-variable prior LLR.
 *
 * Conventions shared by every entry point
 *   - Status: every function returns SAGMS_OK (0) or a negative SAGMS_E*
 *     code; sagms_last_error() then holds a message (thread-local).  No
 *     function aborts or throws across the ABI.
 *   - Bit vectors are packed in uint64 words: bit b of word w is index
 *     64 w + b; unused high bits of the last word are written as zero.
 *     A per-frame vector of nbits bits occupies words(nbits) = ceil(nbits/64)
 *     consecutive words; frame f of a batch starts at word f * words(nbits).
 *   - Device buffers are caller-owned device pointers (hipMalloc'd or torch
 *     tensors) on the current HIP device; `stream` is a hipStream_t passed
 *     as void* (NULL = the null stream).  Every device call is asynchronous
 *     on `stream` and never synchronises.  Host pointers are named *_host.
 *   - A graph handle is immutable after it is built and may be shared by
 *     calls on several streams at once.  Its device tables are copied to the
 *     current HIP device when it is built (if the process has a device), and
 *     to another device by sagms_graph_upload.  The device calls
 *     (sagms_gen_errors, sagms_decode, sagms_decode_soft, sagms_judge)
 *     allocate nothing, copy nothing and never synchronise: they only launch
 *     kernels, so they may be captured into a HIP graph, first call
 *     included.  Decoder gains are evaluated inside the kernels.
 */
#ifndef SAGMS_H
#define SAGMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SAGMS_OK 0
#define SAGMS_EINVAL (-1)       /* bad argument (null pointer, size, range)  */
#define SAGMS_ENOMEM (-2)       /* host or device allocation failed          */
#define SAGMS_EUNSUPPORTED (-3) /* graph shape outside the compiled kernels   */
#define SAGMS_EHIP (-4)         /* a HIP runtime call failed                  */

/* ---- decoder selection ----------------------------------------------- */
typedef enum {
    SAGMS_MS = 0,    /* min-sum, eq. (ms_cn)                                */
    SAGMS_SMS = 1,   /* min-sum scaled by a fixed alpha (Section II)        */
    SAGMS_SAGMS = 2, /* syndrome-adaptive gain, eqs. (alphaeff), (sagms_cn) */
    SAGMS_BP = 3     /* belief propagation, eq. (bp4_cn) (comparison)       */
} sagms_kind;

/* Message-passing schedule.
 *   FLOODING  Algorithm 1: every check updates from the previous round's
 *             variable messages, then every variable.
 *   LAYERED   (not in the paper; this library's reading) the checks are
 *             split into layers of checks with pairwise disjoint supports,
 *             by first fit in ascending check index, and a round visits the
 *             layers in order: each check of a layer takes v2c = posterior
 *             - its own previous output (FP32), computes its output by the
 *             same check rule and gains as FLOODING, and sets posterior =
 *             v2c + new output, so later layers see earlier layers' updates
 *             within the round (the kernel may run checks of several
 *             layers in one pass when every variable still meets its checks
 *             in layer order, which gives the same results).  Gains, hard
 *             decisions, the residual test
 *             and the round count are as in FLOODING (gains from the
 *             residual syndrome at the start of the round).  MS, SMS and
 *             SAGMS with FP32 messages, sagms_decode / sagms_decode_soft
 *             only, on graphs the flooding decoder supports whose checks
 *             all have degree 6, 8 or 10 (SAGMS_EUNSUPPORTED otherwise).
 *             Unscaled MS can overflow FP32 on frames that never converge;
 *             IEEE infinities and NaNs then follow (a NaN posterior
 *             decides 0).  frames_per_wave is ignored. */
typedef enum { SAGMS_FLOODING = 0, SAGMS_LAYERED = 1 } sagms_schedule;

/* Message formats (posteriors are always FP32 sums of the messages):
 *   FP32  FP32 messages; BP evaluates its CN in FP64
 *   FP16  every v2c / c2v message saturated to +-65504 and rounded to IEEE
 *         half (nearest even): v2c = half(posterior - c2v), CN output =
 *         sign * half(gain * min) with the product in FP32
 *   INT6  sign + 6-bit magnitude on a grid of step 1/4 (+-15.75): q(x) =
 *         clamp(nearest-even(4x), -63, 63) / 4 for every message and for
 *         the prior, so posterior sums are exact
 * FP16 / INT6 apply to MS, SMS and SAGMS (SAGMS_EUNSUPPORTED for BP). */
typedef enum {
    SAGMS_MSG_FP32 = 0,
    SAGMS_MSG_FP16 = 1,
    SAGMS_MSG_INT6 = 2
} sagms_msg_precision;

/* Decoder configuration (Algorithm 1 inputs besides H, s and L0).
 *   lmax       maximum number of CN/VN update rounds, >= 1
 *   alpha      SMS scale, in (0, 1]
 *   alpha_min, alpha_max, eta
 *              SAGMS gain law of eq. (alphaeff): per round,
 *              g = alpha_max - (alpha_max - alpha_min) * w / m with w the
 *              weight of the residual syndrome and m the number of checks,
 *              times eta at unsatisfied checks.  0 < alpha_min, alpha_max
 *              <= 1, eta >= 1, and the stability constraint of Section III,
 *              alpha_max * eta <= 1, is enforced (SAGMS_EINVAL otherwise).
 * Fields not used by `kind` are ignored. */
typedef struct {
    int32_t kind;          /* sagms_kind          */
    int32_t schedule;      /* sagms_schedule      */
    int32_t lmax;
    int32_t msg_precision; /* sagms_msg_precision */
    double alpha;
    double alpha_min;
    double alpha_max;
    double eta;
    int32_t frames_per_wave; /* launch shape: frames decoded one after the other by
                                one wavefront.  1..1024: that many for every
                                wavefront.  0 (library default): a tapered
                                launch, 16 per wavefront, with the frames at
                                the end of the batch in runs of 8, 4, 2 and 1
                                so that the last wavefronts finish together.
                                Results do not depend on it */
    int32_t reserved;        /* must be 0 */
} sagms_decoder_cfg;

typedef struct sagms_graph_s* sagms_graph;

typedef struct {
    int32_t m, n;          /* checks, variables of the decoding matrix H      */
    int32_t n_edges;       /* number of ones of H (Tanner-graph edges)        */
    int32_t k;             /* logical dimension n - rank H - rank H_other, or
                              -1 when no other matrix was given              */
    int32_t dc_max, dv_max;/* largest check / variable degree                 */
    int32_t words_n;       /* ceil(n / 64): words per error plane (ex, ez)    */
    int32_t words_m;       /* ceil(m / 64): words per syndrome frame          */
    int32_t joint;         /* 1 for a joint graph (sagms_build_gb_joint)      */
    int32_t words_e;       /* words per estimate frame: words_n, or 2 words_n
                              (x part, then z part) for a joint graph         */
    int32_t layered_group; /* SAGMS_LAYERED: lanes per frame: 8 .. 64, or 1
                              for the matrix compiled into the one-lane
                              kernel (the l = 63 GB code's H_Z, rows in
                              sagms_build_gb's order); 0 when the layered
                              schedule cannot run the graph              */
    int32_t layered_passes;/* SAGMS_LAYERED: passes per round, one check per
                              lane of a group in each (m for the one-lane
                              kernel: a lane updates every check in turn);
                              0 likewise                                  */
} sagms_graph_info_t;

/* ---- graphs (host only; no device needed) ----------------------------- */

/* Tanner graph of a binary check matrix H (m x n) given in CSR form on the
 * host: the ones of row i are col_idx[row_ptr[i] .. row_ptr[i+1]-1].
 * Section II notation: check i has neighbours M(i), variable j has N(j).
 * The optional other CSS matrix (m_other rows, same n) is used only by the
 * logical judge; pass m_other = 0 and NULL pointers to omit it.
 * Requirements: 1 <= m, 1 <= n <= 4096, column indices in [0, n), no
 * repeated column in a row, every check degree >= 2 (SAGMS_EINVAL), and
 * H * H_other^T = 0 over GF(2) when H_other is given (SAGMS_EINVAL).
 * The handle is owned by the library: release it with sagms_destroy_graph. */
int sagms_build_graph(int32_t m, int32_t n, const int32_t* row_ptr_host, const int32_t* col_idx_host,
                      int32_t m_other, const int32_t* row_ptr_other_host,
                      const int32_t* col_idx_other_host, sagms_graph* out);

/* The GB code of circulant size l with polynomials a(x), b(x) given by their
 * exponent lists (values in [0, l), distinct; Section II: the generalized
 * bicycle family).  Circulant convention A[i][j] = 1 iff (j - i) mod l is an
 * exponent of a.  Builds the decoding matrix H = H_Z = [B^T | A^T] and the
 * other matrix H_X = [A | B], so that X errors are decoded from their H_Z
 * syndrome.  n = 2l, m = l.  The decoder's FP32 posterior of a variable sums
 * its checks in the order of the polynomial terms as given: variable i < l
 * meets checks (i + b_t) mod l for t = 0, 1, ..., variable l + i meets
 * (i + a_t) mod l (sagms_build_graph: ascending check index). */
int sagms_build_gb(int32_t l, const int32_t* a_host, int32_t wa, const int32_t* b_host, int32_t wb,
                   sagms_graph* out);

/* Joint (quaternary) graph of the same GB code, for decoding X and Z errors
 * together as the paper's own decoders do (Section II's quaternary Tanner
 * graph; Section V setup: the [[126,28]] code on the overcomplete m = 126
 * matrix, d_c = d_v = |a| + |b|).  m = 2l check rows over n = 2l qubits:
 * rows 0 .. l-1 are the rows of H_X = [A | B] with Pauli X on their support
 * (X-type), rows l .. 2l-1 the rows of H_Z = [B^T | A^T] with Pauli Z
 * (Z-type).  Syndromes hold m bits: bit i < l is H_X e_z, bit l + i is
 * H_Z e_x (the symplectic product of row and error).  Estimates hold
 * words_e = 2 words_n words per frame: x_hat, then z_hat.  Decoded by
 * sagms_decode / sagms_decode_soft (flooding; MS, SMS, SAGMS; FP32 messages)
 * and judged by sagms_judge_joint; not accepted by batches, the server, the
 * layered schedule or sagms_judge.  The posterior sums of variable i < l
 * take its X-type checks (i - a_t) mod l, then its Z-type checks
 * l + (i + b_t) mod l; variable l + i the X-type checks (i - b_t) mod l,
 * then the Z-type checks l + (i + a_t) mod l, each in term order. */
int sagms_build_gb_joint(int32_t l, const int32_t* a_host, int32_t wa, const int32_t* b_host, int32_t wb,
                         sagms_graph* out);

int sagms_graph_info(sagms_graph g, sagms_graph_info_t* info);

/* Copies the decoding matrix H as packed rows: row i occupies words_e words
 * starting at rows_host + i * words_e (joint graphs: the row's x part, then
 * its z part; an X-type row has its support in the z part, since it detects
 * the Z part of an error). */
int sagms_graph_rows(sagms_graph g, uint64_t* rows_host);

/* Copies the logical basis used by the judge: k rows of words_n words, a
 * basis of ker(H_other) modulo rowspace(H).  Joint graphs: 2k rows of
 * words_e words (u | v), such that a residual (r_x | r_z) is a logical error
 * iff u.r_x + v.r_z is odd for some row: rows 0 .. k-1 are the Z-type
 * logicals ker(H_X) mod rowspace(H_Z) as (z | 0), rows k .. 2k-1 the X-type
 * logicals ker(H_Z) mod rowspace(H_X) as (0 | x). */
int sagms_graph_logicals(sagms_graph g, uint64_t* rows_host);

int sagms_destroy_graph(sagms_graph g);

/* Copies the graph's device tables (edge and LDS address tables, packed
 * rows, logical basis, layered schedule tables; a few KB) to the current HIP
 * device, once: later calls on that device return SAGMS_OK at once.  The
 * graph builders already do this for the device current when they run.
 * Synchronous (hipMalloc + hipMemcpy); not for use under stream capture.
 * The device calls return SAGMS_EINVAL on a device without the tables.
 * The copies are freed by sagms_destroy_graph. */
int sagms_graph_upload(sagms_graph g);

/* Binary prior LLR of the X part of a depolarizing error of strength p:
 * ln((1 - 2p/3) / (2p/3)) (the binary marginal of the prior of Section II),
 * rounded to float.  Returns NaN for p outside (0, 0.75). */
float sagms_prior_llr(double p);

/* Prior log-ratio of a joint graph's variables for the depolarizing channel
 * of strength p: L0 = ln((1 - p) / (p / 3)), the same against X, Y and Z
 * (Section II's L0 with e0 = p), rounded to float.  NaN for p outside
 * (0, 0.75). */
float sagms_depolarizing_llr(double p);

/* BP-matching ratio of eq. (alphastar): the scale that makes the min-sum
 * check output equal the BP output when all d_c - 1 incoming magnitudes
 * equal L0, (2 / L0) atanh(tanh(L0 / 2)^(d_c - 1)), evaluated in double
 * without cancellation for large L0.  NaN unless L0 > 0 and d_c >= 2. */
double sagms_alpha_star(double l0, int32_t dc);

/* Derived SAGMS gains (Corollary 1 with the ratio of the Section V setup):
 * alpha_max = alpha*(L0, d_c), alpha_min = ratio * alpha_max, and eta =
 * 1 / alpha_max (the largest value with alpha_max * eta <= 1, Section III)
 * when eta <= 0, else the given eta.  Writes kind = SAGMS and the three
 * gains into *cfg, leaving its other fields unchanged.  SAGMS_EINVAL unless
 * L0 > 0, d_c >= 2, 0 < ratio <= 1 and alpha_max * eta <= 1. */
int sagms_derive_gains(double l0, int32_t dc, double ratio, double eta, sagms_decoder_cfg* cfg);

/* ---- device entry points --------------------------------------------- */

/* Depolarizing errors and their syndromes (Section II, channel and syndrome).
 * For frames frame0 .. frame0 + nframes - 1 and qubits q < n: one
 * Philox4x32-10 block (Salmon et al., SC'11) with key (seed mod 2^32,
 * seed >> 32) and counter (q / 4, frame mod 2^32, frame >> 32, stream_id)
 * gives 32-bit word u = output[q mod 4]; with T_X = floor(p/3 * 2^32),
 * T_Y = floor((2p)/3 * 2^32), T_Z = floor(p * 2^32) (IEEE double), the Pauli
 * is X if u < T_X, Y if u < T_Y, Z if u < T_Z, else I.
 * Outputs (device, packed): ex, ez [nframes][words_n] the X and Z parts
 * (ez may be NULL to skip it, except for a joint graph), synd
 * [nframes][words_m] = H e_x (mod 2), or for a joint graph the symplectic
 * syndrome (H_X e_z, H_Z e_x).
 * 0 <= p < 1; 0 <= nframes <= 2^31 - 1 (0 is a no-op; SAGMS_EINVAL outside,
 * checked before any device work, as for every device call). */
int sagms_gen_errors(sagms_graph g, uint64_t seed, uint32_t stream_id, uint64_t frame0, int64_t nframes,
                     double p, uint64_t* ex, uint64_t* ez, uint64_t* synd, void* stream);

/* Decode nframes syndromes (Algorithm 1, flooding schedule).
 *   synd      device [nframes][words_m] packed syndromes s (bits at or above
 *             m in the last word of a frame are ignored)
 *   llr0      device [n] float prior LLRs L0_j (finite; -0.0 reads as +0.0)
 *   ehat      device [nframes][words_n] packed hard decisions e_hat
 *   iters     device [nframes] number of CN update rounds performed:
 *             0 if the first hard decision [L0 < 0] already satisfies s,
 *             the round at which the residual syndrome became zero, or lmax
 *   converged device [nframes] 1 iff s xor H e_hat = 0
 * Each round: gains from the residual syndrome, CN update (eq. (ms_cn),
 * scaled per eq. (alphaeff)/(sagms_cn), or eq. (bp4_cn) for BP), VN update
 * (eq. (bp4_vn)), hard decision e_j = [posterior_j < 0], residual syndrome,
 * exit when it is zero.  Messages are FP32; each posterior is summed in
 * its graph's check order (see the two graph builders) and v2c =
 * posterior - c2v; the BP CN runs in FP64.
 * Per-frame results do not depend on nframes, the batch split or the
 * stream.  0 <= nframes <= 2^31 - 1. */
int sagms_decode(sagms_graph g, const uint64_t* synd, const float* llr0, const sagms_decoder_cfg* cfg,
                 int64_t nframes, uint64_t* ehat, int32_t* iters, uint8_t* converged, void* stream);

/* sagms_decode plus soft output: posterior (device, float [nframes][n],
 * row f at posterior + f * n) receives every variable's last posterior
 * L0_j + sum of its incoming c2v messages (the quantity whose sign is the
 * hard decision of Algorithm 1).  Same status codes as sagms_decode. */
int sagms_decode_soft(sagms_graph g, const uint64_t* synd, const float* llr0, const sagms_decoder_cfg* cfg,
                      int64_t nframes, uint64_t* ehat, int32_t* iters, uint8_t* converged, float* posterior,
                      void* stream);

/* On a joint graph (sagms_build_gb_joint) the same two calls decode X and Z
 * together with scalar messages:
 *   llr0      device [n] float: L0_j = ln(P(I) / P(W)), the same for W = X,
 *             Y, Z (Section II's depolarizing prior ln((1 - e0) / (e0 / 3)))
 *   ehat      device [nframes][2 words_n]: x_hat words, then z_hat words
 *   posterior device float [nframes][n][3]: the last beliefs Gamma^X,
 *             Gamma^Y, Gamma^Z of every variable
 * Each variable's beliefs are Gamma^X = L0 + S_Z, Gamma^Z = L0 + S_X,
 * Gamma^Y = L0 + (S_X + S_Z), with S_X (S_Z) the FP32 sum of its X-type
 * (Z-type) checks' outputs in the builder's order; the message to a check
 * of Pauli P is min over the two Paulis A that anticommute with P of
 * (Gamma^A - that check's own output) - min(0, Gamma^P) (the min-sum form of
 * the log-domain scalar BP4 reduction the paper's Section I footnote cites);
 * the hard decision is the argmin over (I, X, Y, Z) of (0, Gamma^X,
 * Gamma^Y, Gamma^Z), first minimum on ties; the residual syndrome is the
 * symplectic product (eq. (resid)); m counts both check types in eq.
 * (synratio).  Check outputs are the min-sum outputs of the binary decoder
 * with magnitudes saturated at 2^64.  MS, SMS and SAGMS with FP32 messages
 * and the flooding schedule (SAGMS_EUNSUPPORTED otherwise). */

/* Logical-failure judge.  Frame f fails iff converged[f] == 0, or the
 * residual r = ex xor ehat has odd overlap with some row of the logical
 * basis (equivalently r is not in the rowspace of H_other; Section II:
 * decoding succeeds when the residual syndrome is zero, and the residual
 * error must be a stabilizer).  Needs a graph built with H_other.
 *   ex, ehat  device [nframes][words_n]; converged, iters device [nframes]
 *   fail      device [nframes] (may be NULL): 1 for a failed frame
 *   counters  device uint64 [2], accumulated with atomics (not cleared):
 *             counters[0] += failures, counters[1] += sum of iters */
int sagms_judge(sagms_graph g, const uint64_t* ex, const uint64_t* ehat, const uint8_t* converged,
                const int32_t* iters, int64_t nframes, uint8_t* fail, uint64_t* counters, void* stream);

/* The judge of a joint graph: frame f fails iff converged[f] == 0 or the
 * residual (ex xor x_hat, ez xor z_hat) anticommutes with a logical operator
 * (a row (u | v) of sagms_graph_logicals has u.r_x + v.r_z odd), i.e. it is
 * not in the stabilizer group.  ex, ez device [nframes][words_n]; ehat
 * device [nframes][2 words_n]; the rest as for sagms_judge.  SAGMS_EINVAL
 * for a graph that is not joint. */
int sagms_judge_joint(sagms_graph g, const uint64_t* ex, const uint64_t* ez, const uint64_t* ehat,
                      const uint8_t* converged, const int32_t* iters, int64_t nframes, uint8_t* fail,
                      uint64_t* counters, void* stream);

/* ---- mixed-code batches ------------------------------------------------
 * A batch decodes, in one call, several runs of frames ("segments"), each of
 * its own code: the same Algorithm 1 as sagms_decode, with one decoder
 * configuration for all segments.  Every frame's outputs equal those of
 * sagms_decode on that segment alone, bit for bit, whatever the plan, the
 * mix or the order in which frames run.  The buffers are bound when the
 * batch is created (device pointers of the device current at creation); the
 * caller refills the syndromes and calls sagms_batch_run again. */

typedef struct sagms_batch_s* sagms_batch;

typedef struct {
    sagms_graph graph;         /* code of the segment                            */
    const uint64_t* synd;      /* device [nframes][words_m]                      */
    const float* llr0;         /* device [n]                                     */
    int64_t nframes;           /* >= 0                                           */
    uint64_t* ehat;            /* device [nframes][words_n]                      */
    int32_t* iters;            /* device [nframes]                               */
    uint8_t* converged;        /* device [nframes]                               */
    float* posterior;          /* device [nframes][n], or NULL                   */
} sagms_segment;

/* How a batch is launched.
 *   SINGLE    one persistent kernel over all segments: waves take tiles of
 *             tile_frames frames from work queues until all are done (the
 *             kernel's registers are those of the largest code's shape)
 *   TIERED    one persistent kernel per register class of the codes, in
 *             stream order from the largest class down
 *   PER_CODE  one sagms_decode launch per segment, tile_frames frames per
 *             wave
 * waves_per_block (1, 2 or 4), blocks_per_cu (0 = as many as fit, else
 * 1..64), reg_budget (0 = the compiler's register allocation, 1 = a
 * tighter one allowing one more resident wave per SIMD for the register
 * classes that have one compiled, the compiler's for the others) and unroll
 * (decoding rounds per iteration of a wave's round loop: 1 or 2, 0 reads as
 * 1; every round keeps its own exit test) apply to the persistent plans; a
 * code class whose LDS slices would exceed 64 KiB per block runs with
 * waves_per_block halved until they fit.  Results never depend on the
 * plan. */
typedef enum { SAGMS_PLAN_SINGLE = 0, SAGMS_PLAN_TIERED = 1, SAGMS_PLAN_PER_CODE = 2 } sagms_plan_kind;

typedef struct {
    int32_t kind;            /* sagms_plan_kind     */
    int32_t tile_frames;     /* 1 .. 1024           */
    int32_t waves_per_block;
    int32_t blocks_per_cu;
    int32_t reg_budget;
    int32_t unroll;          /* 0, 1 or 2           */
} sagms_plan;

typedef struct {
    sagms_plan plan;
    float ms;                /* median time of one run, milliseconds */
} sagms_tune_result;

/* Creates a batch of nseg (1..16) segments for decoder cfg (MS, SMS or
 * SAGMS with the flooding schedule; BP or SAGMS_LAYERED is
 * SAGMS_EUNSUPPORTED).  Checks every argument (SAGMS_EINVAL),
 * uploads the graphs' tables to the current device and synchronizes it.
 * The initial plan is SINGLE with tile_frames 8, waves_per_block 4,
 * blocks_per_cu 0, reg_budget 0 and unroll 1.  The batch keeps its own copy of cfg
 * and of the segment table; the graphs must outlive it. */
int sagms_batch_create(const sagms_segment* segs, int32_t nseg, const sagms_decoder_cfg* cfg, sagms_batch* out);

/* Replaces the plan (checked as described at sagms_plan; SAGMS_EINVAL) and
 * drops an instantiated graph. */
int sagms_batch_set_plan(sagms_batch b, const sagms_plan* plan);
int sagms_batch_get_plan(sagms_batch b, sagms_plan* plan);

/* Enqueues one decode of every segment on `stream` (NULL = the null
 * stream): the instantiated graph if there is one, else the plan's kernels.
 * Calls that overlap in time on one batch race on its work queues: order
 * them on one stream. */
int sagms_batch_run(sagms_batch b, void* stream);

/* Captures the current plan's launches (queue reset and kernels, no memset
 * or copy nodes) into a HIP graph and instantiates it; later
 * sagms_batch_run calls launch the graph.  Host call, not stream-ordered. */
int sagms_batch_instantiate(sagms_batch b);

/* Autotuner: times every candidate plan (SINGLE, and TIERED when the codes
 * fall in more than one register class, with tile_frames in {4, 8, 16, 32},
 * waves_per_block in {1, 2, 4}, unroll in {1, 2} and both register budgets
 * where they differ; PER_CODE with tile_frames in {4, 8, 16, 32}) on the
 * batch's own buffers, `reps` (1..100) timed runs each after one warm-up
 * run, keeps the plan with the smallest median time and returns it in *best
 * (may be NULL).
 * Up to `cap` results go to results (may be NULL), their number to *count
 * (may be NULL).  The runs overwrite the batch's outputs; the stream is
 * synchronized on return. */
int sagms_batch_tune(sagms_batch b, void* stream, int32_t reps, sagms_tune_result* results, int32_t cap,
                     int32_t* count, sagms_plan* best);

int sagms_batch_destroy(sagms_batch b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one decode
 * of nseg (1..16) segments, as sagms_batch_create + sagms_batch_run with
 * `plan` (NULL = the initial plan of a batch: SINGLE, tile_frames 8,
 * waves_per_block 4, unroll 1), without a batch object.  Same checks and status codes
 * as sagms_batch_create and sagms_batch_set_plan; every frame's outputs equal
 * those of sagms_decode on that segment alone, bit for bit.
 *   Allocates nothing: no hipMalloc or hipFree, no host-to-device copy.  The
 *   persistent launches' work-queue counters live in a library-owned static
 *   device array of 16 KiB per device (4 register classes x 16 queues),
 *   held until the process ends and reset by a kernel at every launch.  Its
 *   address is taken when a graph is first uploaded to the device, so the
 *   graphs must have their tables on the current device (SAGMS_EINVAL
 *   otherwise).  More segments than 16 are refused (SAGMS_EINVAL).
 *   The array is shared by every call on a device: calls that overlap in
 *   time on one device (on different streams, or from several threads) race
 *   on it and must be ordered by the caller, e.g. on one stream.  The
 *   PER_CODE plan uses no queue counters. */
int sagms_decode_segments(const sagms_segment* segs, int32_t nseg, const sagms_decoder_cfg* cfg,
                          const sagms_plan* plan, void* stream);

/* ---- serving ----------------------------------------------------------
 * Continuous batching of decode requests (Algorithm 1 on each request's
 * frames, one decoder configuration, several codes).  Requests wait in one
 * FIFO per register class of the codes.  Each progress step first retires
 * finished launches (their outputs are copied to the requests' host buffers
 * and their completions recorded), then, while one of the server's streams
 * is free, takes the class whose oldest waiting request is oldest among the
 * classes ready to launch (min_launch_frames waiting; or max_wait_us
 * exceeded while fewer than half of the streams, rounded up, are busy; or
 * no launch in flight) and admits requests from it in order
 * while the launch holds at most
 * max_frames_per_launch frames and all launches in flight at most
 * max_frames_in_flight frames (the device-memory budget); the admitted
 * frames go to the GPU as one copy, one persistent mixed-code launch and one
 * copy back, on that stream.  Launches on different streams overlap on the
 * device, so requests that arrive while others run are admitted as soon as a
 * stream and budget are free.  Every frame's outputs equal those of
 * sagms_decode on that frame alone.  A server is used from one host thread. */

typedef struct sagms_server_s* sagms_server;

typedef struct {
    int64_t max_frames_in_flight;  /* frames in all launches in flight, >= max_frames_per_launch */
    int32_t max_frames_per_launch; /* 1 .. 2^24; also the largest request    */
    int32_t min_launch_frames;     /* a class is launched once it has this many
                                      frames waiting (0 .. max_frames_per_launch), */
    double max_wait_us;            /* or once its oldest request has waited this
                                      long (>= 0) while fewer than half of the
                                      streams are busy, or at once when
                                      nothing is in flight                    */
    int32_t streams;               /* launches in flight at once, 1 .. 8     */
    int32_t tile_frames;           /* persistent-kernel tile, 1 .. 1024      */
    int32_t waves_per_block;       /* 1, 2 or 4 (halved where LDS needs it)  */
    int32_t reg_budget;            /* 0 or 1, as in sagms_plan               */
} sagms_server_cfg;

typedef struct {
    int32_t code;                /* index of the graph given at creation          */
    int32_t nframes;             /* 1 .. max_frames_per_launch                    */
    const uint64_t* synd;        /* host [nframes][words_m]; read at admission    */
    uint64_t* ehat;              /* host [nframes][words_n]                       */
    int32_t* iters;              /* host [nframes]                                */
    uint8_t* converged;          /* host [nframes]                                */
    double deadline_us;          /* cancel if not admitted within this many us
                                    after submission; 0 = no deadline             */
} sagms_request;

enum { SAGMS_REQ_DONE = 0, SAGMS_REQ_CANCELLED = 1 };

typedef struct {
    int64_t id;                  /* as returned by sagms_server_submit            */
    int32_t status;              /* SAGMS_REQ_DONE or SAGMS_REQ_CANCELLED         */
    int32_t reserved;
    double submit_us;            /* server clock (us since creation)              */
    double admit_us;             /* when its launch was enqueued (-1: cancelled)  */
    double done_us;              /* when the host saw its launch finish           */
} sagms_completion;

/* Creates a server for ncodes (1..16) graphs with host prior vectors
 * llr0_host[c] (float [n_c], copied), decoder cfg (MS, SMS or SAGMS, flooding
 * schedule; SAGMS_EUNSUPPORTED otherwise) and
 * serving configuration scfg, on the current device.  Allocates its streams,
 * pinned staging and device buffers (in all: streams x max_frames_per_launch
 * frames of syndromes and outputs) and synchronizes the device. */
int sagms_server_create(const sagms_graph* graphs, const float* const* llr0_host, int32_t ncodes,
                        const sagms_decoder_cfg* cfg, const sagms_server_cfg* scfg, sagms_server* out);

/* Queues a request (checked: SAGMS_EINVAL).  Its host buffers must stay
 * valid until its completion has been returned.  *id may be NULL. */
int sagms_server_submit(sagms_server s, const sagms_request* req, int64_t* id);

/* One progress step (retire, then admit and launch; never blocks), then
 * returns up to cap completions in order of completion.  A launch that
 * cannot be enqueued returns its error and leaves its requests queued, in
 * their order (the step then waits for that stream). */
int sagms_server_progress(sagms_server s, sagms_completion* done, int32_t cap, int32_t* ndone);

/* Requests waiting, frames in launches in flight, completions not yet returned. */
int sagms_server_pending(sagms_server s, int64_t* queued, int64_t* frames_in_flight, int64_t* completions);

/* Open-loop trace replay on an idle server: request i is submitted when
 * arrival_us[i] (non-decreasing) microseconds have passed since the call
 * began, with that scheduled time as its submission time; progress steps
 * run until every request has completed, and out[i] receives request i's
 * completion.  Returns SAGMS_EHIP if no launch finishes for timeout_s. */
int sagms_server_replay(sagms_server s, const sagms_request* reqs, const double* arrival_us, int64_t n,
                        double timeout_s, sagms_completion* out);

/* Waits for the server's streams, then frees everything it holds. */
int sagms_server_destroy(sagms_server s);

/* Message for the last non-zero status returned on this thread. */
const char* sagms_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SAGMS_H */
