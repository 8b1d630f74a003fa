// Internal declarations of libsagms (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sagms.h"

namespace sagms {

// ---- errors -----------------------------------------------------------
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
#define SAGMS_HIP(call)                                      \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, #call);    \
    } while (0)

constexpr int kMaxDevices = 64;
constexpr int kMaxN = 4096;
// Frames per device call: at most 2^31 - 1, which keeps every launch's grid
// (at most one wavefront per frame) within 2^31 - 1 blocks.
constexpr int64_t kMaxFramesPerCall = 0x7fffffffLL;
// SAGMS_OK, or SAGMS_EINVAL for nframes < 0 or > kMaxFramesPerCall (host
// check, before any device work).
int check_frames(int64_t nframes);

// ---- decode kernel shapes ---------------------------------------------
// One wavefront decodes one frame at a time.  Lane l owns checks l + 64 k
// (k < CPL) and variables l + 64 k (k < VPL).  DC / DV bound the check and
// variable degrees (shorter rows are padded).
struct DecodeShape {
    int dc, dv, cpl, vpl;
};

// Every compiled shape, X(index, DC, DV, CPL, VPL), in increasing order of
// register use: a mixed-code kernel compiled for shapes 0..HI holds the
// registers of shape HI (see kMixedTiers).
#define SAGMS_DECODE_SHAPES(X) \
    X(0, 4, 2, 1, 1)           \
    X(1, 6, 3, 1, 1)           \
    X(2, 10, 5, 1, 2)          \
    X(3, 16, 8, 1, 2)          \
    X(4, 10, 5, 2, 4)          \
    X(5, 6, 3, 4, 8)           \
    X(6, 16, 8, 2, 4)          \
    X(7, 8, 4, 4, 8)           \
    X(8, 10, 5, 8, 16)
constexpr int kNumShapes = 9;
// Highest shape index of each mixed-kernel tier: the tiers share one
// occupancy class each (shapes 0-2 fit 64 VGPRs, 3-4 fit 128, 5-7 fit 168).
constexpr int kMixedTiers[] = {2, 4, 7, 8};
constexpr int kNumMixedTiers = 4;
// Index of a shape in SAGMS_DECODE_SHAPES, or -1.
int shape_index(const DecodeShape& s);

// Per-wave LDS layout of the decode kernels, in 32-bit words:
//   c2v slots  [dc][cw]   slot(c, p) = p * cw + c  (cw = 64 * cpl)
//   zero       [64] words holding 0.0f (padding of short variables)
//   posterior  [64 * vpl] posterior of variable j at post0 + j
//   padpost    [64] words holding +inf (padding of short checks)
//   gains      [2 * (64 * cpl + 1)] pairs (gain satisfied, gain unsatisfied)
//              indexed by the residual-syndrome weight w; only when cpl > 1
//              (one-block codes keep the table in registers)
// The padding lanes of one half-wavefront of an LDS gather all read one word
// of a padding pool, chosen in a bank that the half's other lanes leave free,
// so that padding adds no bank conflict (place_padding, lds_pad.h).
struct DecodeLayout {
    int cw, zero, post0, padpost, gain0, words;
};

// Joint (quaternary) decode kernels: shapes X(index, DC, DV, CPL, VPL) with
// DV = 2 * DVH, ranks [0, DVH) of a variable being its X-type checks and
// [DVH, DV) its Z-type checks (shorter halves padded).
#define SAGMS_JOINT_SHAPES(X) \
    X(0, 4, 4, 1, 1)          \
    X(1, 6, 6, 1, 1)          \
    X(2, 10, 10, 2, 2)        \
    X(3, 10, 10, 4, 4)
constexpr int kNumJointShapes = 4;

// Per-wave LDS layout of the joint kernel, in 32-bit words:
//   c2v slots  [dc][cw]        slot(c, p) = p * cw + c  (cw = 64 * cpl)
//   zero       [64]            0.0f (padding of short variable halves)
//   pairx      [64 * vpl] x 2  (A, W) of variable j for its X-type checks
//   pairz      [64 * vpl] x 2  (A, W) of variable j for its Z-type checks
//   padpair    [64] x 2        (+inf, +0) (padding of short checks)
//   gains      [2 * (cw + 1)]  gain pairs by residual weight
struct JointLayout {
    int cw, zero, pairx, pairz, padpair, gain0, words;
};

// Gain law of a decoder configuration (eq. (alphaeff)): kind MS / BP (gain
// 1), SMS (alpha), SAGMS (alpha_min, alpha_max, eta).  The kernels evaluate
// it per residual weight w in IEEE double, operation by operation, and round
// to float (gain_pair, decode_core.h), so no table is allocated per call.
struct GainLaw {
    int32_t kind;
    int32_t pad;
    double a, amin, amax, eta;
};

// Layered schedule (layered.hip, layers.cpp): the checks in layers of checks
// with disjoint supports (first fit in ascending check index), every layer
// cut into passes of at most `group` checks; a wavefront decodes 64 / group
// frames, one per group of `group` lanes.  LDS words per wavefront: the
// shared tables (pass table, variable pairs, gains, prior, the prior's
// residual bits), then per frame
// the posteriors (npad words), each check's outputs in compressed form (4
// words per check) and the syndrome and residual bits (2 * wm words each).
// Schedules of at most this many passes keep each lane's check outputs in
// registers (layered.hip; a second, shorter register form serves schedules
// of at most kLayeredRegPassesShort passes); longer ones keep them in LDS.
constexpr int kLayeredRegPasses = 24;
constexpr int kLayeredRegPassesShort = 16;

// Host part of the layered plan, computed when the graph is built; status
// is SAGMS_OK when the layered schedule can run the graph, else the code
// returned by a layered decode, with `why` as its message.
struct LayeredHost {
    int status = SAGMS_EUNSUPPORTED;
    std::string why;
    int dc = 0, group = 0, passes = 0, npad = 0, group_words = 0, table_words = 0;
    bool regs = false;  // check outputs in registers (passes <= kLayeredRegPasses)
    std::vector<int32_t> pass_check;   // [passes][group], -1 = idle lane
    std::vector<uint32_t> check_vars;  // [m][dc / 2] variable pairs as 16-bit byte offsets 4 j
};

struct LayeredPlan {
    int dc = 0, group = 0, passes = 0, npad = 0, group_words = 0, table_words = 0;
    bool regs = false;
    int32_t* pass_check = nullptr;   // device copy of LayeredHost::pass_check
    uint32_t* check_vars = nullptr;  // device copy of LayeredHost::check_vars
};

// Device copies of a graph's tables on one HIP device, created by
// upload_tables (graph build, sagms_graph_upload, batch and server set-up)
// and never on a decode, sampling or judge call.
struct DeviceTables {
    bool ready = false;
    LayeredPlan layered;           // valid when the graph's LayeredHost status is SAGMS_OK
    uint32_t* cn_addr = nullptr;   // [cpl * dc][64] LDS word index of the posterior read at (check, pos)
    uint32_t* vn_addr = nullptr;   // [vpl * dv][64] LDS word index of the c2v slot read at (var, rank)
    int32_t* cols = nullptr;       // [m][dc_max] column of (check, pos), -1 padded (sampler)
    uint64_t* rows = nullptr;      // [m][words_n] packed rows of H (sampler)
    uint64_t* logicals = nullptr;  // [k][words_n]
};

struct Graph {
    int m = 0, n = 0, E = 0, dc_max = 0, dv_max = 0, k = -1, wn = 0, wm = 0;
    // joint graph: checks 0 .. m/2 - 1 are X-type rows (Pauli X), the rest
    // Z-type rows (Pauli Z); error and estimate vectors are (x | z) halves of
    // wn words each (we = 2 wn words); rows_bits is [m][we]; logicals holds
    // 2k rows (u | v) whose parity u.r_x + v.r_z flags a logical failure
    bool joint = false;
    int we = 0;
    int dvh = 0;  // joint: the larger of a variable's X-type and Z-type degrees
    // decoding matrix H: row i has columns cols[row_ptr[i] .. row_ptr[i+1]-1] in
    // the order used as the check's edge positions
    std::vector<int> row_ptr, cols;
    std::vector<uint64_t> rows_bits;   // [m][wn]
    std::vector<uint64_t> logicals;    // [k][wn]
    bool have_other = false;
    // GB codes: circulant size and exponents (term order of the polynomials)
    bool is_gb = false;
    int gb_l = 0;
    std::vector<int> gb_a, gb_b;
    // every variable's (check, position) pairs in the order of its posterior sum
    std::vector<std::vector<std::pair<int, int>>> var_edges;
    bool shape_ok = false;
    DecodeShape shape{};
    DecodeLayout layout{};
    std::vector<uint32_t> cn_addr_host, vn_addr_host;
    JointLayout jlayout{};  // joint graphs
    LayeredHost layered;
    std::mutex mu;
    DeviceTables dev[kMaxDevices];
};

// GF(2) helpers (graph.cpp)
int gf2_rank(std::vector<uint64_t> rows, int nrows, int wn);

// Creates the device tables of g on the current device (once; later calls
// return them).  Allocates and copies synchronously: set-up calls only.
int upload_tables(Graph* g, DeviceTables** out);
// The device tables of g on the current device; SAGMS_EINVAL if they were
// never uploaded there.  Allocates nothing.
int device_tables(Graph* g, DeviceTables** out);
// Layered plan of g computed on the host (layers.cpp), stored in g->layered.
void plan_layers(Graph* g);

// Shape selection for the decode kernels.
bool pick_shape(int m, int n, int dc, int dv, DecodeShape* out);
DecodeLayout make_layout(const DecodeShape& s);

// Shape selection for the joint kernels; layout of a joint shape.
bool pick_joint_shape(int m, int n, int dc, int dvh, DecodeShape* out);
JointLayout make_joint_layout(const DecodeShape& s);

// Arguments of the joint decode kernel.
struct JointArgs {
    const uint64_t* synd;
    const float* llr0;
    GainLaw gains;
    const uint32_t* cn_addr;  // [cpl * dc][64] LDS word index of the (A, W) pair read at (check, pos)
    const uint32_t* vn_addr;  // [vpl * dv][64] LDS word index of the c2v slot read at (var, rank)
    uint64_t* ehat;           // [nframes][2 wn]: x-hat words, then z-hat words
    int32_t* iters;
    uint8_t* conv;
    float* gamma;             // optional [nframes][n][3] last beliefs (X, Y, Z)
    int64_t nframes;
    int m, n, wm, wn, lmax, frames_per_wave;
    JointLayout L;
};
int launch_joint(const DecodeShape& s, const JointArgs& a, hipStream_t st);
// Waves of a kernel resident on the current device (occupancy x compute
// units), queried once per kernel and device (decode.hip).
int resident_waves(const void* kernel, int wpb, size_t lds, int64_t* out);

// Kernel launchers (one translation unit each).
struct DecodeArgs {
    const uint64_t* synd;
    const float* llr0;
    GainLaw gains;       // per-round gains by residual weight (gain_pair)
    const uint32_t* cn_addr;
    const uint32_t* vn_addr;
    uint64_t* ehat;
    int32_t* iters;
    uint8_t* conv;
    float* post;  // optional soft output [nframes][n]
    int64_t nframes;
    int m, n, wm, wn, lmax, frames_per_wave;
    DecodeLayout L;
};
int launch_decode(const DecodeShape& s, bool bp, int msg_precision, const DecodeArgs& a, hipStream_t st);
int launch_layered(const LayeredPlan& plan, const DecodeArgs& a, hipStream_t st);

constexpr int kDecodeFramesPerWave = 16;  // frames per wave before the taper
constexpr int kMixedTileFrames = 8;       // default tile of a mixed-code batch
// Decoder configuration checks (api.cpp); SAGMS_OK or a status.
int check_cfg(const sagms_decoder_cfg* c);
// Gain law of a configuration (checked by check_cfg).
GainLaw gain_law(const sagms_decoder_cfg* cfg);
// Kernel arguments of one decode call (frames_per_wave 0 = default).
DecodeArgs decode_args(const Graph* g, const DeviceTables* t, const GainLaw& gains, const uint64_t* synd,
                       const float* llr0, int64_t nframes, uint64_t* ehat, int32_t* iters, uint8_t* converged,
                       float* posterior, int lmax, int frames_per_wave);

// ---- mixed-code persistent decode ---------------------------------------
// A batch holds up to kMaxSegments segments, each a run of frames of one
// code.  The frames are cut into tiles of tile_frames frames; the tiles of
// all segments, in segment order, are dealt round-robin to nq queues (tile t
// to queue t mod nq, as its (t div nq)-th entry).  A wave starts on queue
// blockIdx mod nq, takes tiles from it with one atomic increment each, and
// moves on to the next queue when it is empty; it exits after finding every
// queue empty once.
constexpr int kMaxSegments = 16;
constexpr int kMaxQueues = 16;
constexpr int kQueueStride = 64;  // 32-bit words between counters (256 B)

struct MixedSegment {
    DecodeArgs a;
    int32_t shape;  // index in SAGMS_DECODE_SHAPES
    int32_t pad;
};

// Passed by value (kernel arguments, about 2.4 KB): the segment table is
// read with scalar loads and is captured with the launch in a HIP graph.
struct MixedArgs {
    MixedSegment segs[kMaxSegments];
    uint32_t* queues;                   // device [nq * kQueueStride], zero at launch
    int64_t tile_end[kMaxSegments];     // tiles of segments 0..s
    int64_t ntiles;
    int nseg, nq, tile_frames, words;   // words: LDS words per wave
};

// LDS words per wave of the mixed kernel of a tier (largest layout in it).
int mixed_words(int tier);
// Whether a tier has a kernel with register budget `budget` (0 = the
// compiler's allocation, 1 = one more resident wave per SIMD).
bool mixed_has_budget(int tier, int budget);
// Resident blocks per CU of a mixed kernel (occupancy of registers and LDS).
int mixed_max_blocks(int tier, int budget, int mt, int unroll, int waves_per_block, int* out);
// Zeroes the queue counters, then launches the persistent kernel (MS / SMS /
// SAGMS; BP has no mixed kernel).
int launch_mixed(int tier, int budget, int mt, int unroll, const MixedArgs& m, int blocks, int waves_per_block,
                 hipStream_t st);

// Register class of a shape index (-1 if none).
int mixed_tier_of_shape(int shape_idx);
// The tight register budget where the tier has one, else the compiler's.
int mixed_budget_of(int tier, int requested);
// Waves per block of a tier: the requested number, halved until the block's
// LDS slices fit 64 KiB.
int mixed_waves_of(int tier, int requested);

// Resident blocks per CU of the mixed kernels, queried once per (tier,
// register budget, message format, waves per block); a fixed table, so that
// lookups never allocate.
struct OccupancyCache {
    int blocks[kNumMixedTiers][2][3][2][5];  // [tier][budget][format][unroll - 1][waves per block]
    OccupancyCache();
    int get(int tier, int budget, int mt, int unroll, int waves_per_block, int* out);
};

struct MixedLaunch {
    int tile_frames, waves_per_block, blocks_per_cu, reg_budget, unroll;
};

// One persistent launch over nseg segments (all of register class <= tier)
// on stream st: grid = resident capacity (capped by blocks_per_cu when > 0,
// and by the number of tiles); queues = this launch's own counter block.
int launch_segments(const MixedSegment* segs, int nseg, int tier, const MixedLaunch& p, int num_cu, int mt,
                    uint32_t* queues, OccupancyCache* occ, hipStream_t st);

// The segments of a mixed-code decode in launch order (register tier
// descending, then lane slots per round descending, then the caller's
// order), with their kernel arguments.  Fixed size: no allocation.
struct SegmentSet {
    int nseg = 0;
    MixedSegment segs[kMaxSegments];
    int tier[kMaxSegments];
    DecodeShape shape[kMaxSegments];
};

// Checks the segments and the configuration (MS, SMS or SAGMS, flooding)
// and fills *out.  upload: copy missing graph tables to the current device
// (set-up calls); otherwise a graph without tables there is an error.
int prepare_segments(const sagms_segment* segs, int nseg, const sagms_decoder_cfg* cfg, bool upload,
                     SegmentSet* out);
// Checks a launch plan (SAGMS_EINVAL).
int check_plan(const sagms_plan* p);
// Enqueues one decode of every segment under plan p: PER_CODE as single-code
// decode launches, SINGLE / TIERED as persistent launches whose tier t uses
// the kMaxQueues counters at queues + t * kMaxQueues * kQueueStride.
int enqueue_segments(const SegmentSet& set, const sagms_plan& p, int mt, int num_cu, uint32_t* queues,
                     OccupancyCache* occ, hipStream_t st);

// Queue counters of sagms_decode_segments: a static device array of
// kNumMixedTiers * kMaxQueues * kQueueStride words (mixed.hip).
constexpr size_t kScratchWords = (size_t)kNumMixedTiers * kMaxQueues * kQueueStride;
// Takes the array's device address on the current device (once per device;
// called from upload_tables, which runs with the device current).
int scratch_setup();
// The array's device address on the current device, set up before.
int scratch_queues(uint32_t** out);


struct SampleArgs {
    const int32_t* cols;
    const uint64_t* rows;
    uint64_t* ex;
    uint64_t* ez;
    uint64_t* synd;
    uint64_t seed;
    uint64_t frame0;
    int64_t nframes;
    uint32_t stream_id;
    uint32_t tx, ty, tz;
    int m, n, dc, wn, wm, frames_per_wave, lanes_per_frame;
    int joint;  // rows / columns over the (x | z) planes: rows of 2 wn words, columns j < n in x, n + j in z
};
int launch_sample(const SampleArgs& a, hipStream_t st);

struct JudgeArgs {
    const uint64_t* ex;
    const uint64_t* ez;  // joint graphs: the Z plane (words wplane .. wn - 1 of the residual); else null
    const uint64_t* ehat;
    const uint8_t* conv;
    const int32_t* iters;
    const uint64_t* logicals;
    uint8_t* fail;
    uint64_t* counters;
    int64_t nframes;
    int k, wn;   // basis rows; words per residual (= per e_hat frame)
    int wplane;  // words per frame of ex (and ez)
};
int launch_judge(const JudgeArgs& a, hipStream_t st);

}  // namespace sagms
