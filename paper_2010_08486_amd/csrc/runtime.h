// Host runtime of the detector: plans, device workspace, launch sequences.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dct.h"
#include "dog.h"
#include "dog_internal.h"

#define DOG_NKERNELS 5

namespace dog {

// ---------------------------------------------------------------- plan
struct Plan {
    dog_params prm;
    int k = 0;      // DoG planes
    int n_g = 0;    // Gaussian planes (k+1)
    std::vector<double> sigma;
    std::vector<int> r;
    std::vector<float> weights;  // per-plane vectors, zero-padded
    std::vector<std::vector<double>> half64;  // per plane: FP64 weights w_j, j = 0..r
    LadderDesc desc;
};

bool validate_params(const dog_params& p, std::string* err);
int build_plan(const dog_params& p, Plan* plan, std::string* err);
bool same_params(const dog_params& a, const dog_params& b);
int dog_planes_for(double smin, double smax, double ratio);

// ---------------------------------------------------------------- prune
double overlap_fraction(int y1, int x1, double s1, int y2, int x2, double s2);
void sort_blobs(std::vector<dog_blob>& v);
void prune_blobs(std::vector<dog_blob>& v, const std::vector<double>& sigma64, double overlap,
                 bool coalesce);
void radius_histogram(const std::vector<double>& ladder, int k, const dog_blob* v, int64_t n,
                      int64_t* counts);

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define DOG_HIP(call)                                  \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess)                          \
            return ::dog::hip_fail(e_, #call);         \
    } while (0)

// ---------------------------------------------------------------- memory
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct PinBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// A frame ready for a launch: device pixels.
struct FrameIn {
    const float* d;
    int H, W;
    long long stride;
};

// Geometry of one tiling variant.
struct Variant {
    int S, NW, BI, BN, NWN;
    int group;   // blur tiles take runs of planes (cost-balanced)
    int band() const { return S * NW * BI; }
    int nms_band() const { return BN * NWN; }
};

// A run of consecutive planes that one blur workgroup takes in turn: top,
// top-1, ..., top-count+1 (widest first); cost in tap chunks.
struct PlaneRun {
    int top, count, cost;
};
// The planes (indices, widest first) cut into runs: one plane each, or
// (group) cost-balanced runs of consecutive planes.
std::vector<PlaneRun> plane_runs(const Plan& P, const std::vector<int>& planes, int S, bool group);

const char* last_error();
int check_image(const void* p, int64_t h, int64_t w, int64_t stride);
int export_blobs(const std::vector<dog_blob>& v, dog_blob** out, int64_t* n);

// Detector on n frames (host or device pixels) with results per frame; see
// dog_detect_batch.
int detect_frames(dog_context* ctx, const dog_params* params, int32_t n_frames,
                  const dog_frame* frames, hipStream_t s, dog_result* results);

}  // namespace dog

// Kernel launchers (kernels.hip).
extern "C" {
int dogk_num_variants();
void dogk_variant_geometry(int v, int* S, int* NW, int* BI, int* BN, int* NWN);
int dogk_variant_ring(int v);
int dogk_variant_group(int v);
hipError_t dogk_launch_pass(int variant, const dog::LaunchArgs* args, int pass, int grid,
                            int fft_logn, int wide1, hipStream_t stream, hipEvent_t* ev);
int dogk_variant_merges_fft(int v, int logn);
hipError_t dogk_launch_nms_ev(int variant, const dog::LaunchArgs* args, int grid3, int debug,
                              hipStream_t stream, hipEvent_t* ev);
hipError_t dogk_launch_nms(int variant, const dog::LaunchArgs* args, int grid3, int max_gauss,
                           int debug, hipStream_t stream);
hipError_t dogk_untranspose(const float* src, float* dst, int n_planes, int H, int W,
                            long long pitch, hipStream_t stream);
hipError_t dogk_fill_u32(uint32_t* p, int n, uint32_t v, hipStream_t stream);
hipError_t dogk_occupancy(int variant, int* wg1, int* wg2, int* wg3);
size_t dogk_preprocess_scratch_bytes();
int dogk_preprocess_max_radius();
hipError_t dogk_preprocess(const float* d_in, int H, int W, long long stride, const float* d_w,
                           int r, float* d_s, float* d_out, void* d_scratch, uint32_t rank_lo,
                           uint32_t rank_hi, hipStream_t stream);
size_t dogk_preprocess_noalloc_bytes();
hipError_t dogk_preprocess_noalloc(const float* d_in, int H, int W, long long stride,
                                   const float* w_host, int r, float* d_s, float* d_out,
                                   float* d_limits, uint32_t rank_lo, uint32_t rank_hi,
                                   hipStream_t stream);
}

struct dog_context {
    int device = 0;
    uint64_t budget = 0;
    uint64_t used = 0;             // bytes allocated on the device
    hipStream_t stream = nullptr;
    int n_cu = 0;
    int variant = 0;               // active kernel variant
    int variant_auto = 0;          // built-in default
    bool variant_forced = false;   // pinned by dog_set_variant
    std::map<std::string, int> tuned;  // "HxW|radii" -> autotuned variant
    std::map<std::string, int> tuned_dct;  // "HxW|radii" -> autotuned transform threshold (taps)
    int occ[3] = {0, 0, 0};        // workgroups per CU of each kernel (active variant)

    // device memory accounting: allocations are checked against `budget`
    // together with the lanes' (child contexts of grouped batches, which
    // share their parent's budget).  exact_alloc: allocate what is asked
    // (server slots, whose every byte is committed by admission) instead of
    // growing buffers by a quarter; room_margin: bytes kept free for tables
    // and candidates when a batch is cut into chunks that fit the budget.
    dog_context* parent = nullptr;
    bool exact_alloc = false;
    uint64_t room_margin = 64ull << 20;

    dog::DevBuf planes;            // T, L (and debug D) planes of all frames
    dog::DevBuf input;             // device copies of host frames
    dog::DevBuf tables;            // frames, ladder, weights, units
    dog::DevBuf cand;              // CandHeader + records
    uint32_t cap = 0;              // record capacity of `cand`

    dog::PinBuf h_tables;          // staging of the launch tables
    dog::PinBuf h_cand;            // readback of header + records
    dog::PinBuf h_ends;            // per local-maximum workgroup: end of its record range
    dog::PinBuf h_input;           // staging of host frames
    dog::DevBuf prep;              // preprocessing: select state, histograms, weights
    dog::DevBuf prn;               // device pruning: FP64 ladder sigmas
    std::vector<double> prn_sig;   // the sigmas `prn` holds
    void* prn_sig_dev = nullptr;   // the buffer they were uploaded to
    dog::PinBuf h_prn;             // device pruning: sigma staging, then the kernel's output
    uint32_t prn_blobs = 0;        // blobs one pruning workgroup holds (from the LDS limit)
    uint32_t prn_pairs = 0;        // touching pairs it holds
    double prep_sigma = -1.0;      // smoothing sigma whose weights `prep` holds
    bool prep_dirty = false;       // `prep` histograms not known to be zero
    hipEvent_t ev_prep = nullptr;  // recorded after the last preprocessing launch

    // optional per-kernel timing: start and end events of each kernel's
    // dispatch, on the stream it is launched on
    bool profiling = false;
    // kernels: pass 1, pass 2, local maxima, then the transform-domain
    // blur's forward 1, forward 2, inverse 1, inverse 2
    hipEvent_t ev[2 * DOG_NKERNELS] = {};
    double kernel_ms[DOG_NKERNELS] = {};
    int64_t kernel_launches = 0;

    // the captured launch sequence of the last table layout (frame table
    // upload, three kernels, readback) and what it was built for
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<long long> graph_key;
    std::vector<long long> seen_key;   // layout of the previous call
    dog::LaunchArgs args;
    dog::FftLaunch fft{};          // transform-domain launches of the current tables
    int n_gauss = 0;
    bool debug_planes = false;     // the current tables write the DoG planes
    bool wide1 = false;            // every frame of the tables allows 16-byte row loads
    std::vector<const int*> frame_rows;  // per frame: pass-1 and pass-2 row tables
    int row_pad = 0;
    size_t frames_bytes = 0;       // frame table bytes uploaded per launch
    uint32_t guess = 0;            // records read back by the captured sequence
    bool tables_ready = false;     // device tables match graph_key
    bool use_graphs = true;        // replay a captured graph (else launch directly)
    hipEvent_t ev_done = nullptr;  // recorded after a sequence; polled for completion

    // a launch not yet collected (dog_detect_device_async): frame count,
    // the one-frame descriptor passed inline, and the stream
    bool pending = false;
    int pend_n = 0;
    bool pend_inline = false;
    dog::FrameDesc pend_f0{};
    hipStream_t pend_stream = nullptr;

    // batches: frames are cut into groups of at most group_pixels pixels,
    // run concurrently on `lane_count` child contexts (each with its own
    // stream and workspace); group_pixels 0 runs a batch as one sequence
    int64_t group_pixels = (int64_t)1 << 20;
    int lane_count = 3;
    std::vector<dog_context*> lanes;
    hipEvent_t ev_fork = nullptr;

    // transform-domain blur: planes whose kernels have at least this many
    // taps, on frames whose sides are powers of two in [64, 4096]; 0: never
    int dct_min_taps = 0;
    bool dct_forced = false;     // dct_min_taps set by dog_set_dct (else the tuned choice per shape)

    bool have_plan = false;
    uint64_t plan_gen = 0;
    // transform-domain tables of the current plan, kept across table
    // rebuilds: per line length the twiddles and post-twiddles, per (line
    // length, plane) the transfer function over N (fp32)
    uint64_t fft_cache_gen = ~0ull;
    std::map<int, std::vector<float>> fft_twiddles;
    std::map<std::pair<int, int>, std::vector<float>> fft_transfer;
    dog::Plan plan;
    uint32_t last_count = 0;       // candidates found by the previous launch (readback guess)
};

namespace dog {

int ctx_alloc(dog_context* c, DevBuf* b, size_t bytes, const char* what);
// Device bytes held by a context and its lanes.
uint64_t ctx_total_used(const dog_context* c);
// Free the workspace buffers of an idle context (planes, inputs, tables,
// candidates); they are allocated again on the next launch.
int ctx_trim(dog_context* c);
// Bytes of a launch sequence over frames of these shapes beyond the planes
// and staged inputs: an upper bound of its launch tables (any variant) and
// the initial candidate buffer.
uint64_t overhead_bound(const Plan& P, int n, const int64_t* heights, const int64_t* widths);
// Bytes the planes (and, for host frames, the staged input) of one frame
// take in a launch sequence, as detect_frames sizes its chunks.
uint64_t frame_plane_bytes(const Plan& P, int64_t H, int64_t W);
uint64_t frame_input_bytes(int64_t H, int64_t W);
int ctx_pin(PinBuf* b, size_t bytes);
int ctx_plan(dog_context* c, const dog_params* prm, const Plan** out);
int ctx_set_variant(dog_context* c, int v);
void drop_graph(dog_context* c);
int choose_variant(const dog_context* c, const std::vector<FrameIn>& frames, const Plan& P);
// Transform threshold (kernel taps; 0 = every plane direct) for frames of
// this shape: the one set by dog_set_dct, else the autotuned one, else 0.
int frame_min_taps(const dog_context* c, int H, int W, const Plan& P);
// Whether frames of this shape can take the transform-domain blur.
bool frame_dct_ok(int H, int W);

// Run the three kernels over `frames` (device pixels) with plan P and read
// back the candidate records, grouped per frame and sorted by (y, x, scale).
// If dbg_D is true the first frame's DoG planes are also written to the
// workspace (debug layout).
int run_frames(dog_context* c, const Plan& P, const std::vector<FrameIn>& frames,
               hipStream_t s, std::vector<std::vector<dog_blob>>* out, bool dbg_D,
               long long* pitch0, float** L0, float** D0);
// The two halves of run_frames: queue the launch sequence on s (returns once
// it is queued and marks the context pending), then wait for it and turn the
// candidate records into sorted blob lists per frame.
int launch_frames(dog_context* c, const Plan& P, const std::vector<FrameIn>& frames,
                  hipStream_t s, bool dbg_D, long long* pitch0, float** L0, float** D0);
int collect_frames(dog_context* c, const Plan& P, std::vector<std::vector<dog_blob>>* out);

const char* last_error();
int check_image(const void* p, int64_t h, int64_t w, int64_t stride);
int export_blobs(const std::vector<dog_blob>& v, dog_blob** out, int64_t* n);

// Detector on n frames (host or device pixels) with results per frame; see
// dog_detect_batch.
int detect_frames(dog_context* ctx, const dog_params* params, int32_t n_frames,
                  const dog_frame* frames, hipStream_t s, dog_result* results);

}  // namespace dog
