// C ABI exports (declared in include/dog.h).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "prune_device.h"
#include "runtime.h"

using namespace dog;

namespace {

constexpr int kDefaultVariant = 8;  // LDS-staged, S = 16, 4 waves, 2 chunks staged

int use_device(dog_context* c)
{
    DOG_HIP(hipSetDevice(c->device));
    return DOG_OK;
}

// Entry points that use a context refuse it while a launch of
// dog_detect_device_async is still to be collected.
int ctx_idle(dog_context* c)
{
    if (c->pending) {
        set_error("a launch of dog_detect_device_async has not been finished");
        return DOG_EBUSY;
    }
    return DOG_OK;
}

// The caller's stream as given: NULL is the null (default) stream, so work
// queued there by the caller, which produced the input, runs first.
hipStream_t pick_stream(dog_context* c, void* stream)
{
    (void)c;
    return static_cast<hipStream_t>(stream);
}

void free_context(dog_context* c)
{
    if (!c)
        return;
    (void)hipSetDevice(c->device);
    if (c->pending && c->ev_done)
        (void)hipEventSynchronize(c->ev_done);
    if (c->ev_prep)
        (void)hipEventSynchronize(c->ev_prep);
    for (dog_context* l : c->lanes)
        free_context(l);
    c->lanes.clear();
    if (c->ev_fork)
        (void)hipEventDestroy(c->ev_fork);
    (void)hipSetDevice(c->device);
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    for (DevBuf* b : {&c->planes, &c->input, &c->tables, &c->cand, &c->prep, &c->prn})
        if (b->p)
            (void)hipFree(b->p);
    for (PinBuf* b : {&c->h_tables, &c->h_cand, &c->h_ends, &c->h_input, &c->h_prn})
        if (b->p)
            (void)hipHostFree(b->p);
    drop_graph(c);
    for (hipEvent_t& e : c->ev)
        if (e)
            (void)hipEventDestroy(e);
    if (c->ev_done)
        (void)hipEventDestroy(c->ev_done);
    if (c->ev_prep)
        (void)hipEventDestroy(c->ev_prep);
    if (c->stream)
        (void)hipStreamDestroy(c->stream);
    delete c;
}

std::mutex g_default_mu;
dog_context* g_default = nullptr;

}  // namespace

extern "C" {

const char* dog_last_error(void) { return dog::last_error(); }

const char* dog_version(void) { return "dog-mi355x 0.3 (gfx950, LDS-staged separable stencil and wave-level cosine-transform kernels)"; }

void dog_blobs_free(dog_blob* blobs) { std::free(blobs); }

void dog_results_free(dog_result* results, int32_t n)
{
    if (!results)
        return;
    for (int32_t i = 0; i < n; ++i) {
        std::free(results[i].blobs);
        results[i].blobs = nullptr;
    }
}

int dog_context_create(int device, uint64_t hbm_budget_bytes, dog_context** ctx)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return DOG_EINVAL;
    }
    *ctx = nullptr;
    int ndev = 0;
    DOG_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) {
        set_error("no such device");
        return DOG_EINVAL;
    }
    std::unique_ptr<dog_context> c(new dog_context());
    c->device = device;
    DOG_HIP(hipSetDevice(device));
    DOG_HIP(hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device));
    size_t free_b = 0, total_b = 0;
    DOG_HIP(hipMemGetInfo(&free_b, &total_b));
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * (double)free_b);
    DOG_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->variant_auto = kDefaultVariant;
    int rc = ctx_set_variant(c.get(), kDefaultVariant);
    if (rc != DOG_OK) {
        free_context(c.release());
        return rc;
    }
    *ctx = c.release();
    return DOG_OK;
}

void dog_context_destroy(dog_context* ctx) { free_context(ctx); }

int dog_num_variants(void) { return dogk_num_variants(); }

int dog_variant_info(int variant, int32_t* S, int32_t* waves, int32_t* strips, int32_t* nms_rows)
{
    if (variant < 0 || variant >= dogk_num_variants()) {
        set_error("no such kernel variant");
        return DOG_EINVAL;
    }
    int s, nw, bi, bn, nwn;
    dogk_variant_geometry(variant, &s, &nw, &bi, &bn, &nwn);
    if (S)
        *S = s;
    if (waves)
        *waves = nw;
    if (strips)
        *strips = bi;
    if (nms_rows)
        *nms_rows = bn;
    return DOG_OK;
}

int dog_set_variant(dog_context* ctx, int variant)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return DOG_EINVAL;
    }
    int rc = ctx_idle(ctx);
    if (rc != DOG_OK)
        return rc;
    rc = use_device(ctx);
    if (rc != DOG_OK)
        return rc;
    if ((rc = ctx_set_variant(ctx, variant)) != DOG_OK)
        return rc;
    ctx->variant_forced = variant >= 0;
    return DOG_OK;
}

int dog_set_profiling(dog_context* ctx, int32_t on)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return DOG_EINVAL;
    }
    if (ctx->pending)
        return ctx_idle(ctx);
    if (ctx->profiling != (on != 0))
        drop_graph(ctx);
    ctx->profiling = on != 0;
    for (double& m : ctx->kernel_ms)
        m = 0.0;
    ctx->kernel_launches = 0;
    return DOG_OK;
}

int dog_set_dct(dog_context* ctx, int32_t min_taps)
{
    if (!ctx || min_taps < -1) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    if (ctx->pending)
        return ctx_idle(ctx);
    const bool forced = min_taps >= 0;
    if (ctx->dct_forced != forced || (forced && ctx->dct_min_taps != min_taps))
        drop_graph(ctx);
    ctx->dct_forced = forced;
    ctx->dct_min_taps = forced ? min_taps : 0;
    return DOG_OK;
}

int dog_kernel_times_all(dog_context* ctx, double* ms_out, int32_t cap, int64_t* launches_out)
{
    if (!ctx || !ms_out || cap < DOG_NKERNELS) {
        set_error("invalid argument (ms_out needs room for 5 kernels)");
        return DOG_EINVAL;
    }
    for (int i = 0; i < DOG_NKERNELS; ++i)
        ms_out[i] = ctx->kernel_ms[i];
    if (launches_out)
        *launches_out = ctx->kernel_launches;
    return DOG_OK;
}

int dog_set_batch_grouping(dog_context* ctx, int64_t max_group_pixels, int32_t lanes)
{
    if (!ctx || max_group_pixels < 0 || lanes < 1 || lanes > 16) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    if (ctx->pending)
        return ctx_idle(ctx);
    ctx->group_pixels = max_group_pixels;
    ctx->lane_count = lanes;
    return DOG_OK;
}

int dog_set_graph_mode(dog_context* ctx, int32_t on)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return DOG_EINVAL;
    }
    if (ctx->pending)
        return ctx_idle(ctx);
    if (ctx->use_graphs != (on != 0))
        drop_graph(ctx);
    ctx->use_graphs = on != 0;
    return DOG_OK;
}

int dog_kernel_times(dog_context* ctx, double* ms_out, int64_t* launches_out)
{
    if (!ctx || !ms_out) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    for (int i = 0; i < 3; ++i)
        ms_out[i] = ctx->kernel_ms[i];
    if (launches_out)
        *launches_out = ctx->kernel_launches;
    return DOG_OK;
}


int dog_prune(const dog_params* params, dog_blob* blobs, int64_t n, int64_t* n_out)
{
    if (!params || !n_out || n < 0 || (n > 0 && !blobs)) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    Plan P;
    std::string err;
    int rc = build_plan(*params, &P, &err);
    if (rc != DOG_OK) {
        set_error(err);
        return rc;
    }
    std::vector<dog_blob> v(blobs, blobs + n);
    for (dog_blob& b : v) {
        if (b.scale < 0 || b.scale >= P.k) {
            set_error("blob scale index outside the ladder");
            return DOG_EINVAL;
        }
        b.sigma = (float)P.sigma[b.scale];
    }
    sort_blobs(v);
    prune_blobs(v, P.sigma, P.prm.overlap, P.prm.coalesce != 0);
    std::copy(v.begin(), v.end(), blobs);
    *n_out = (int64_t)v.size();
    return DOG_OK;
}

int dog_prune_device(dog_context* ctx, const dog_params* params, const dog_blob* d_blobs,
                     int64_t n, void* stream, dog_blob** blobs_out, int64_t* count_out,
                     int64_t* hist_out)
{
    if (!ctx || !params || !blobs_out || !count_out || n < 0 || (n > 0 && !d_blobs)) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    *blobs_out = nullptr;
    *count_out = 0;
    int rc = ctx_idle(ctx);
    if (rc != DOG_OK)
        return rc;
    if ((rc = use_device(ctx)) != DOG_OK)
        return rc;
    const Plan* P = nullptr;
    if ((rc = ctx_plan(ctx, params, &P)) != DOG_OK)
        return rc;
    const hipStream_t st = pick_stream(ctx, stream);
    if (ctx->prn_blobs == 0) {
        // the workgroup's capacity follows the LDS one workgroup may use
        int lds = 0;
        DOG_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                      ctx->device));
        ctx->prn_blobs = 4096;
        ctx->prn_pairs = 8192;
        while (ctx->prn_blobs > 256 &&
               dogk_prune_lds_bytes(ctx->prn_blobs, ctx->prn_pairs) + 4096 > (size_t)lds) {
            ctx->prn_blobs /= 2;
            ctx->prn_pairs /= 2;
        }
    }
    const size_t sig_bytes = sizeof(double) * (size_t)P->n_g;
    const size_t out_bytes = sizeof(PruneHead) + sizeof(dog_blob) * (size_t)ctx->prn_blobs;
    if (ctx->prn.bytes < sig_bytes)
        ctx->prn_sig_dev = nullptr;   // the buffer is replaced: upload the ladder again
    if ((rc = ctx_alloc(ctx, &ctx->prn, sig_bytes, "pruning ladder")) != DOG_OK)
        return rc;
    // pinned: the ladder's staging, then the kernel's output (written by the
    // kernel straight into host memory)
    const size_t head_off = (sig_bytes + 255) & ~(size_t)255;
    if ((rc = ctx_pin(&ctx->h_prn, head_off + out_bytes)) != DOG_OK)
        return rc;
    char* h = static_cast<char*>(ctx->h_prn.p);
    PruneHead* head = reinterpret_cast<PruneHead*>(h + head_off);
    std::vector<dog_blob> v;
    std::vector<int64_t> hist(P->k, 0);
    bool on_host = n > (int64_t)ctx->prn_blobs;
    if (!on_host) {
        if (ctx->prn_sig_dev != ctx->prn.p || ctx->prn_sig != P->sigma) {
            // a new ladder (or buffer): staged, then copied in stream order
            DOG_HIP(hipStreamSynchronize(st));   // the staging area is reused
            std::memcpy(h, P->sigma.data(), sig_bytes);
            DOG_HIP(hipMemcpyAsync(ctx->prn.p, h, sig_bytes, hipMemcpyHostToDevice, st));
            ctx->prn_sig = P->sigma;
            ctx->prn_sig_dev = ctx->prn.p;
        }
        head->status = 0;
        PruneArgs a{};
        a.cand = nullptr;
        a.recs = d_blobs;
        a.cap = (uint32_t)n;
        a.n_direct = (uint32_t)n;
        a.sig64 = static_cast<const double*>(ctx->prn.p);
        a.sig_max = P->sigma[P->k - 1];
        a.overlap = P->prm.overlap;
        a.k = P->k;
        a.coalesce = P->prm.coalesce;
        a.blob_in = 1;
        a.max_blobs = ctx->prn_blobs;
        a.max_pairs = ctx->prn_pairs;
        a.out = reinterpret_cast<char*>(head);
        a.out_stride = out_bytes;
        DOG_HIP(dogk_prune(&a, 1, st));
        DOG_HIP(hipStreamSynchronize(st));
        if (head->status == kPruneBadRecord) {
            set_error("blob outside 0 <= y, x < 32768 or scale outside the ladder");
            return DOG_EINVAL;
        }
        if (head->status == kPruneDone) {
            const dog_blob* ob = reinterpret_cast<const dog_blob*>(head + 1);
            v.assign(ob, ob + head->n_out);
            for (int i = 0; i < P->k; ++i)
                hist[i] = head->hist[i];
        } else if (head->status == kPruneTooManyPairs) {
            on_host = true;
        } else {
            set_error("device pruning did not complete");
            return DOG_EDEVICE;
        }
    }
    if (on_host) {
        // more than one workgroup holds: the same steps on the host
        v.resize((size_t)n);
        DOG_HIP(hipMemcpyAsync(v.data(), d_blobs, sizeof(dog_blob) * (size_t)n,
                               hipMemcpyDeviceToHost, st));
        DOG_HIP(hipStreamSynchronize(st));
        for (dog_blob& b : v) {
            if (b.scale < 0 || b.scale >= P->k || b.y < 0 || b.y > 32767 || b.x < 0 ||
                b.x > 32767) {
                set_error("blob outside 0 <= y, x < 32768 or scale outside the ladder");
                return DOG_EINVAL;
            }
            b.sigma = (float)P->sigma[b.scale];
        }
        sort_blobs(v);
        prune_blobs(v, P->sigma, P->prm.overlap, P->prm.coalesce != 0);
        radius_histogram(P->sigma, P->k, v.data(), (int64_t)v.size(), hist.data());
    }
    if (hist_out)
        std::copy(hist.begin(), hist.end(), hist_out);
    return export_blobs(v, blobs_out, count_out);
}

int dog_radius_histogram(const dog_params* params, const dog_blob* blobs, int64_t n,
                         int64_t* counts_out)
{
    if (!params || !counts_out || n < 0 || (n > 0 && !blobs)) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    Plan P;
    std::string err;
    const int rc = build_plan(*params, &P, &err);
    if (rc != DOG_OK) {
        set_error(err);
        return rc;
    }
    for (int64_t b = 0; b < n; ++b)
        if (!std::isfinite(blobs[b].sigma)) {
            set_error("blob sigma is not finite");
            return DOG_EINVAL;
        }
    radius_histogram(P.sigma, P.k, blobs, n, counts_out);
    return DOG_OK;
}

int dog_plan_info(const dog_params* params, int32_t* k_out, double* sigmas_out,
                  int32_t* radii_out, int32_t cap)
{
    if (!params || !k_out) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    Plan P;
    std::string err;
    int rc = build_plan(*params, &P, &err);
    if (rc != DOG_OK) {
        set_error(err);
        return rc;
    }
    *k_out = P.k;
    if (cap >= P.n_g) {
        for (int i = 0; i < P.n_g; ++i) {
            if (sigmas_out)
                sigmas_out[i] = P.sigma[i];
            if (radii_out)
                radii_out[i] = P.r[i];
        }
    }
    return DOG_OK;
}

int dog_footprint(const dog_params* params, int32_t n_frames, const int64_t* heights,
                  const int64_t* widths, uint64_t* bytes_out)
{
    if (!params || !bytes_out || n_frames < 0 || (n_frames > 0 && (!heights || !widths))) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    Plan P;
    std::string err;
    int rc = build_plan(*params, &P, &err);
    if (rc != DOG_OK) {
        set_error(err);
        return rc;
    }
    uint64_t planes = 0, input = 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        if (heights[f] < 1 || widths[f] < 1) {
            set_error("frame shapes must be positive");
            return DOG_EINVAL;
        }
        planes += frame_plane_bytes(P, heights[f], widths[f]);
        input += frame_input_bytes(heights[f], widths[f]);  // staged host frame
    }
    auto page = [](uint64_t x) { return (x + 4095) & ~(uint64_t)4095; };
    *bytes_out = page(planes) + page(input) +
                 (n_frames ? overhead_bound(P, n_frames, heights, widths) : 0);
    return DOG_OK;
}

int dog_detect_device(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                      int64_t row_stride, const dog_params* params, void* stream,
                      dog_blob** blobs_out, int64_t* count_out)
{
    if (!ctx || !blobs_out || !count_out) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    *blobs_out = nullptr;
    *count_out = 0;
    int rc = check_image(d_image, height, width, row_stride);
    if (rc != DOG_OK)
        return rc;
    if ((rc = ctx_idle(ctx)) != DOG_OK)
        return rc;
    if ((rc = use_device(ctx)) != DOG_OK)
        return rc;
    const Plan* P = nullptr;
    if ((rc = ctx_plan(ctx, params, &P)) != DOG_OK)
        return rc;
    std::vector<FrameIn> fr{{d_image, (int)height, (int)width, (long long)row_stride}};
    std::vector<std::vector<dog_blob>> res;
    rc = run_frames(ctx, *P, fr, pick_stream(ctx, stream), &res, false, nullptr, nullptr, nullptr);
    if (rc != DOG_OK)
        return rc;
    prune_blobs(res[0], P->sigma, P->prm.overlap, P->prm.coalesce != 0);
    return export_blobs(res[0], blobs_out, count_out);
}

int dog_detect_device_async(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                            int64_t row_stride, const dog_params* params, void* stream)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return DOG_EINVAL;
    }
    int rc = check_image(d_image, height, width, row_stride);
    if (rc != DOG_OK)
        return rc;
    if ((rc = ctx_idle(ctx)) != DOG_OK)
        return rc;
    if ((rc = use_device(ctx)) != DOG_OK)
        return rc;
    const Plan* P = nullptr;
    if ((rc = ctx_plan(ctx, params, &P)) != DOG_OK)
        return rc;
    std::vector<FrameIn> fr{{d_image, (int)height, (int)width, (long long)row_stride}};
    return launch_frames(ctx, *P, fr, pick_stream(ctx, stream), false, nullptr, nullptr, nullptr);
}

int dog_detect_device_finish(dog_context* ctx, dog_blob** blobs_out, int64_t* count_out)
{
    if (!ctx || !blobs_out || !count_out) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    *blobs_out = nullptr;
    *count_out = 0;
    if (!ctx->pending) {
        set_error("no launch of dog_detect_device_async to finish");
        return DOG_EINVAL;
    }
    int rc = use_device(ctx);
    if (rc != DOG_OK) {
        ctx->pending = false;
        return rc;
    }
    std::vector<std::vector<dog_blob>> res;
    if ((rc = collect_frames(ctx, ctx->plan, &res)) != DOG_OK)
        return rc;
    prune_blobs(res[0], ctx->plan.sigma, ctx->plan.prm.overlap, ctx->plan.prm.coalesce != 0);
    return export_blobs(res[0], blobs_out, count_out);
}

// Arguments of both preprocessing entry points; sets *r to the smoothing
// radius.
static int check_preprocess(const float* d_image, int64_t height, int64_t width,
                            int64_t row_stride, double smooth_sigma, double saturated,
                            const float* d_out, int* r)
{
    if (!d_out) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    const int rc = check_image(d_image, height, width, row_stride);
    if (rc != DOG_OK)
        return rc;
    if (!std::isfinite(smooth_sigma) || smooth_sigma < 0.0 || !(saturated >= 0.0) ||
        !(saturated < 1.0)) {
        set_error("smooth_sigma must be finite and >= 0, saturated in [0, 1)");
        return DOG_EINVAL;
    }
    *r = smooth_sigma > 0.0 ? (int)std::floor(4.0 * smooth_sigma + 0.5) : 0;
    if (*r > dogk_preprocess_max_radius()) {
        set_error("smoothing radius above " + std::to_string(dogk_preprocess_max_radius()));
        return DOG_EINVAL;
    }
    return DOG_OK;
}

// The detector's kernel rule for the smoothing weights: exp(-j^2 / (2 s^2))
// in FP64, normalised over the truncated support, rounded once to fp32 (no
// smoothing: the single weight 1).  wf: 2r+1 floats (r <= 16; no heap use,
// so the entry point that allocates nothing can call it).
static void smoothing_weights(double smooth_sigma, int r, float* wf)
{
    double g[2 * 16 + 1];
    double total = r > 0 ? 0.0 : 1.0;
    g[r] = 1.0;
    for (int j = -r; r > 0 && j <= r; ++j)
        total += (g[j + r] = std::exp(-((double)j * j) / (2.0 * smooth_sigma * smooth_sigma)));
    for (int j = 0; j <= 2 * r; ++j)
        wf[j] = (float)(g[j] / total);
}

// Ranks of the two limits: m = floor(saturated N / 2), at most (N-1)/2.
static void limit_ranks(int64_t height, int64_t width, double saturated, uint32_t* lo,
                        uint32_t* hi)
{
    const long long N = (long long)height * width;
    long long m = (long long)std::floor(saturated * (double)N / 2.0);
    m = std::min(m, (N - 1) / 2);
    *lo = (uint32_t)m;
    *hi = (uint32_t)(N - 1 - m);
}

int dog_preprocess(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                   int64_t row_stride, double smooth_sigma, double saturated, float* d_out,
                   float* d_smoothed, float* limits_out, void* stream)
{
    if (!ctx) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    int r = 0;
    int rc = check_preprocess(d_image, height, width, row_stride, smooth_sigma, saturated, d_out,
                              &r);
    if (rc != DOG_OK)
        return rc;
    if ((rc = ctx_idle(ctx)) != DOG_OK)
        return rc;
    if ((rc = use_device(ctx)) != DOG_OK)
        return rc;
    const size_t scratch = dogk_preprocess_scratch_bytes();
    void* const had = ctx->prep.p;
    if ((rc = ctx_alloc(ctx, &ctx->prep, scratch + 64 * sizeof(float), "preprocessing scratch")) !=
        DOG_OK)
        return rc;
    if (ctx->prep.p != had) {
        // fresh scratch: the kernels expect zero histograms (each call
        // leaves them zero for the next)
        ctx->prep_dirty = true;
        ctx->prep_sigma = -1.0;
    }
    float* d_w = reinterpret_cast<float*>(static_cast<char*>(ctx->prep.p) + scratch);
    hipStream_t st = pick_stream(ctx, stream);
    // the scratch is the context's: a call on another stream first waits
    // (on the device) for the previous call to be done with it
    if (!ctx->ev_prep)
        DOG_HIP(hipEventCreateWithFlags(&ctx->ev_prep, hipEventDisableTiming));
    else
        DOG_HIP(hipStreamWaitEvent(st, ctx->ev_prep, 0));
    if (ctx->prep_dirty) {
        // ordered on this stream after the previous call (the first call of
        // a context, or the one after a failed launch)
        DOG_HIP(hipMemsetAsync(ctx->prep.p, 0, scratch, st));
        ctx->prep_dirty = false;
    }
    if (ctx->prep_sigma != smooth_sigma) {
        float wf[2 * 16 + 1];
        smoothing_weights(smooth_sigma, r, wf);
        DOG_HIP(hipMemcpyAsync(d_w, wf, (size_t)(2 * r + 1) * sizeof(float), hipMemcpyHostToDevice,
                               st));
        DOG_HIP(hipStreamSynchronize(st));
        ctx->prep_sigma = smooth_sigma;
    }
    uint32_t rank_lo = 0, rank_hi = 0;
    limit_ranks(height, width, saturated, &rank_lo, &rank_hi);
    float* d_s = d_smoothed ? d_smoothed : d_out;
    const hipError_t le = dogk_preprocess(d_image, (int)height, (int)width, (long long)row_stride,
                                          d_w, r, d_s, d_out, ctx->prep.p, rank_lo, rank_hi, st);
    if (le != hipSuccess) {
        // some kernels may have run and left counts behind: the next call
        // clears the scratch first, after what was queued here
        ctx->prep_dirty = true;
        (void)hipEventRecord(ctx->ev_prep, st);
        DOG_HIP(le);
    }
    DOG_HIP(hipEventRecord(ctx->ev_prep, st));
    if (limits_out) {
        DOG_HIP(hipMemcpyAsync(limits_out, static_cast<char*>(ctx->prep.p) + 16, 2 * sizeof(float),
                               hipMemcpyDeviceToHost, st));
        DOG_HIP(hipStreamSynchronize(st));
    }
    return DOG_OK;
}

int dog_preprocess_noalloc(const float* d_image, int64_t height, int64_t width,
                           int64_t row_stride, double smooth_sigma, double saturated,
                           float* d_out, float* d_smoothed, float* d_limits, void* stream)
{
    int r = 0;
    const int rc = check_preprocess(d_image, height, width, row_stride, smooth_sigma, saturated,
                                    d_out, &r);
    if (rc != DOG_OK)
        return rc;
    float wf[2 * 16 + 1];
    smoothing_weights(smooth_sigma, r, wf);
    uint32_t rank_lo = 0, rank_hi = 0;
    limit_ranks(height, width, saturated, &rank_lo, &rank_hi);
    DOG_HIP(dogk_preprocess_noalloc(d_image, (int)height, (int)width, (long long)row_stride,
                                    wf, r, d_smoothed ? d_smoothed : d_out, d_out,
                                    d_limits, rank_lo, rank_hi, static_cast<hipStream_t>(stream)));
    return DOG_OK;
}

int dog_debug_candidates(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                         int64_t row_stride, const dog_params* params, dog_blob** blobs_out,
                         int64_t* count_out)
{
    if (!ctx || !blobs_out || !count_out) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    *blobs_out = nullptr;
    *count_out = 0;
    int rc = check_image(d_image, height, width, row_stride);
    if (rc != DOG_OK)
        return rc;
    if ((rc = ctx_idle(ctx)) != DOG_OK)
        return rc;
    if ((rc = use_device(ctx)) != DOG_OK)
        return rc;
    const Plan* P = nullptr;
    if ((rc = ctx_plan(ctx, params, &P)) != DOG_OK)
        return rc;
    std::vector<FrameIn> fr{{d_image, (int)height, (int)width, (long long)row_stride}};
    std::vector<std::vector<dog_blob>> res;
    rc = run_frames(ctx, *P, fr, ctx->stream, &res, false, nullptr, nullptr, nullptr);
    if (rc != DOG_OK)
        return rc;
    return export_blobs(res[0], blobs_out, count_out);
}

int dog_debug_planes(dog_context* ctx, const float* d_image, int64_t height, int64_t width,
                     int64_t row_stride, const dog_params* params, float* L_out, float* D_out,
                     int32_t* k_out)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return DOG_EINVAL;
    }
    int rc = check_image(d_image, height, width, row_stride);
    if (rc != DOG_OK)
        return rc;
    if ((rc = ctx_idle(ctx)) != DOG_OK)
        return rc;
    if ((rc = use_device(ctx)) != DOG_OK)
        return rc;
    const Plan* P = nullptr;
    if ((rc = ctx_plan(ctx, params, &P)) != DOG_OK)
        return rc;
    std::vector<FrameIn> fr{{d_image, (int)height, (int)width, (long long)row_stride}};
    std::vector<std::vector<dog_blob>> res;
    long long pitch = 0;
    float* L = nullptr;
    float* D = nullptr;
    rc = run_frames(ctx, *P, fr, ctx->stream, &res, true, &pitch, &L, &D);
    if (rc != DOG_OK)
        return rc;
    if (L_out)
        DOG_HIP(dogk_untranspose(L, L_out, P->n_g, (int)height, (int)width, pitch, ctx->stream));
    if (D_out)
        DOG_HIP(dogk_untranspose(D, D_out, P->k, (int)height, (int)width, pitch, ctx->stream));
    DOG_HIP(hipStreamSynchronize(ctx->stream));
    if (k_out)
        *k_out = P->k;
    return DOG_OK;
}

int dog_detect_batch(dog_context* ctx, int32_t n_frames, const dog_frame* frames,
                     const dog_params* params, void* stream, dog_result* results)
{
    if (!ctx || n_frames < 0 || (n_frames > 0 && (!frames || !results))) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    const int rc = ctx_idle(ctx);
    if (rc != DOG_OK)
        return rc;
    return detect_frames(ctx, params, n_frames, frames, pick_stream(ctx, stream), results);
}

int dog_detect(const float* image, int64_t height, int64_t width, int64_t row_stride,
               double sigma_min, double sigma_max, double sigma_ratio, double threshold,
               double overlap, dog_blob** blobs_out, int64_t* count_out)
{
    if (!blobs_out || !count_out) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    *blobs_out = nullptr;
    *count_out = 0;
    int rc = check_image(image, height, width, row_stride);
    if (rc != DOG_OK)
        return rc;
    dog_params prm{sigma_min, sigma_max, sigma_ratio, threshold, overlap, 4.0};
    std::string err;
    if (!validate_params(prm, &err)) {
        set_error(err);
        return DOG_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_default_mu);
    if (!g_default) {
        if ((rc = dog_context_create(0, 0, &g_default)) != DOG_OK)
            return rc;
    }
    dog_context* c = g_default;
    if ((rc = use_device(c)) != DOG_OK)
        return rc;
    const size_t bytes = (size_t)height * (size_t)width * sizeof(float);
    if ((rc = ctx_pin(&c->h_input, bytes)) != DOG_OK)
        return rc;
    if ((rc = ctx_alloc(c, &c->input, bytes, "input frame")) != DOG_OK)
        return rc;
    float* hp = static_cast<float*>(c->h_input.p);
    for (int64_t y = 0; y < height; ++y)
        std::memcpy(hp + y * width, image + y * row_stride, (size_t)width * sizeof(float));
    DOG_HIP(hipMemcpyAsync(c->input.p, hp, bytes, hipMemcpyHostToDevice, c->stream));
    // the detector runs on the stream of the upload, after it
    return dog_detect_device(c, static_cast<const float*>(c->input.p), height, width, width, &prm,
                             c->stream, blobs_out, count_out);
}

}  // extern "C"
