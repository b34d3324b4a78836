// C ABI exports (declared in include/dog.h).
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>

#include "runtime.h"

namespace dog {
const char* last_error();
}

using namespace dog;

namespace {

constexpr int kMaxSide = 32768;
constexpr int kDefaultVariant = 0;  // S = 12, R = 4: fastest on 1024x1024 frames

int check_image(const void* p, int64_t h, int64_t w, int64_t stride)
{
    if (!p) {
        set_error("image pointer is NULL");
        return DOG_EINVAL;
    }
    if (h < 1 || w < 1 || h > kMaxSide || w > kMaxSide) {
        set_error("image height and width must be in [1, 32768]");
        return DOG_EINVAL;
    }
    if (stride < w) {
        set_error("row_stride must be >= width");
        return DOG_EINVAL;
    }
    // every plane is addressed with 32-bit byte offsets: input rows and
    // transposed planes (width rows of height rounded up to 64) stay < 2 GiB
    if ((double)h * (double)stride >= (double)(1LL << 29) ||
        (double)w * (double)(h + 63) >= (double)(1LL << 29)) {
        set_error("height * row_stride and width * (height + 63) must be < 2^29");
        return DOG_EINVAL;
    }
    return DOG_OK;
}

int use_device(dog_context* c)
{
    DOG_HIP(hipSetDevice(c->device));
    return DOG_OK;
}

hipStream_t pick_stream(dog_context* c, void* stream)
{
    return stream ? static_cast<hipStream_t>(stream) : c->stream;
}

// Copy a sorted, pruned blob vector into a malloc'd array.
int export_blobs(const std::vector<dog_blob>& v, dog_blob** out, int64_t* n)
{
    *out = nullptr;
    *n = 0;
    if (v.empty())
        return DOG_OK;
    dog_blob* p = static_cast<dog_blob*>(std::malloc(sizeof(dog_blob) * v.size()));
    if (!p) {
        set_error("out of host memory");
        return DOG_ENOMEM;
    }
    std::memcpy(p, v.data(), sizeof(dog_blob) * v.size());
    *out = p;
    *n = (int64_t)v.size();
    return DOG_OK;
}

void free_context(dog_context* c)
{
    if (!c)
        return;
    (void)hipSetDevice(c->device);
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    for (DevBuf* b : {&c->planes, &c->input, &c->tables, &c->cand})
        if (b->p)
            (void)hipFree(b->p);
    for (PinBuf* b : {&c->h_tables, &c->h_cand, &c->h_input})
        if (b->p)
            (void)hipHostFree(b->p);
    drop_graph(c);
    for (hipEvent_t& e : c->ev)
        if (e)
            (void)hipEventDestroy(e);
    if (c->ev_in)
        (void)hipEventDestroy(c->ev_in);
    if (c->stream)
        (void)hipStreamDestroy(c->stream);
    delete c;
}

std::mutex g_default_mu;
dog_context* g_default = nullptr;

}  // namespace

extern "C" {

const char* dog_last_error(void) { return dog::last_error(); }

const char* dog_version(void) { return "dog-mi355x 0.1 (gfx950, persistent separable-stencil kernels)"; }

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
    int rc = use_device(ctx);
    if (rc != DOG_OK)
        return rc;
    return ctx_set_variant(ctx, variant);
}

int dog_set_profiling(dog_context* ctx, int32_t on)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return DOG_EINVAL;
    }
    if (ctx->profiling != (on != 0))
        drop_graph(ctx);
    ctx->profiling = on != 0;
    for (double& m : ctx->kernel_ms)
        m = 0.0;
    ctx->kernel_launches = 0;
    return DOG_OK;
}

int dog_set_graph_mode(dog_context* ctx, int32_t on)
{
    if (!ctx) {
        set_error("ctx is NULL");
        return DOG_EINVAL;
    }
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
    prune_blobs(v, P.sigma, P.prm.overlap);
    std::copy(v.begin(), v.end(), blobs);
    *n_out = (int64_t)v.size();
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
    uint64_t b = 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        const uint64_t pitch = ((uint64_t)heights[f] + 63) / 64 * 64;
        b += 2ull * P.n_g * (uint64_t)widths[f] * pitch * sizeof(float);
        b += (uint64_t)heights[f] * (uint64_t)widths[f] * sizeof(float);  // staged input
    }
    b += 4096ull * (3 * (uint64_t)n_frames * P.n_g + 64) / 64;  // tables (rough, generous)
    *bytes_out = b;
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
    prune_blobs(res[0], P->sigma, P->prm.overlap);
    return export_blobs(res[0], blobs_out, count_out);
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
    for (int32_t f = 0; f < n_frames; ++f)
        std::memset(&results[f], 0, sizeof(dog_result));
    int rc = use_device(ctx);
    if (rc != DOG_OK)
        return rc;
    const Plan* P = nullptr;
    if ((rc = ctx_plan(ctx, params, &P)) != DOG_OK) {
        for (int32_t f = 0; f < n_frames; ++f)
            results[f].status = rc;
        return rc;
    }
    hipStream_t s = pick_stream(ctx, stream);
    int first_err = DOG_OK;
    std::string first_msg;

    // valid frames, and the bytes each needs: planes + staged host pixels
    std::vector<int> idx;
    std::vector<uint64_t> need;
    for (int32_t f = 0; f < n_frames; ++f) {
        const dog_frame& fr = frames[f];
        const int e = check_image(fr.data, fr.height, fr.width, fr.row_stride);
        if (e != DOG_OK) {
            results[f].status = e;
            if (first_err == DOG_OK) {
                first_err = e;
                first_msg = dog::last_error();
            }
            continue;
        }
        const uint64_t pitch = ((uint64_t)fr.height + 63) / 64 * 64;
        uint64_t b = 2ull * P->n_g * (uint64_t)fr.width * pitch * sizeof(float) + 256;
        if (!fr.on_device)
            b += (uint64_t)fr.height * (uint64_t)fr.width * sizeof(float) + 256;
        idx.push_back(f);
        need.push_back(b);
    }
    // consecutive chunks that fit in what the budget leaves for planes and inputs
    const uint64_t fixed = ctx->used - ctx->planes.bytes - ctx->input.bytes;
    const uint64_t room = ctx->budget > fixed + (64u << 20) ? ctx->budget - fixed - (64u << 20) : 0;
    size_t i = 0;
    while (i < idx.size()) {
        size_t j = i;
        uint64_t sum = 0;
        while (j < idx.size() && (j == i || sum + need[j] <= room)) {
            sum += need[j];
            ++j;
        }
        if (sum > room) {
            for (size_t q = i; q < j; ++q)
                results[idx[q]].status = DOG_ENOMEM;
            if (first_err == DOG_OK) {
                first_err = DOG_ENOMEM;
                first_msg = "frame footprint exceeds the HBM budget";
            }
            i = j;
            continue;
        }
        // stage host frames
        uint64_t in_bytes = 0;
        for (size_t q = i; q < j; ++q)
            if (!frames[idx[q]].on_device)
                in_bytes += ((uint64_t)frames[idx[q]].height * frames[idx[q]].width * sizeof(float) + 255) / 256 * 256;
        if (in_bytes) {
            if ((rc = ctx_pin(&ctx->h_input, in_bytes)) != DOG_OK ||
                (rc = ctx_alloc(ctx, &ctx->input, in_bytes, "input frames")) != DOG_OK)
                goto chunk_fail;
        }
        {
            std::vector<FrameIn> fin;
            uint64_t o = 0;
            for (size_t q = i; q < j; ++q) {
                const dog_frame& fr = frames[idx[q]];
                if (fr.on_device) {
                    fin.push_back({fr.data, (int)fr.height, (int)fr.width, (long long)fr.row_stride});
                } else {
                    char* hp = static_cast<char*>(ctx->h_input.p) + o;
                    for (int64_t y = 0; y < fr.height; ++y)
                        std::memcpy(hp + (size_t)y * fr.width * sizeof(float), fr.data + y * fr.row_stride,
                                    (size_t)fr.width * sizeof(float));
                    fin.push_back({reinterpret_cast<const float*>(static_cast<char*>(ctx->input.p) + o),
                                   (int)fr.height, (int)fr.width, (long long)fr.width});
                    o += ((uint64_t)fr.height * fr.width * sizeof(float) + 255) / 256 * 256;
                }
            }
            if (o) {
                hipError_t e = hipMemcpyAsync(ctx->input.p, ctx->h_input.p, o, hipMemcpyHostToDevice, s);
                if (e != hipSuccess) {
                    rc = hip_fail(e, "hipMemcpyAsync(input)");
                    goto chunk_fail;
                }
            }
            std::vector<std::vector<dog_blob>> res;
            rc = run_frames(ctx, *P, fin, s, &res, false, nullptr, nullptr, nullptr);
            if (rc != DOG_OK)
                goto chunk_fail;
            for (size_t q = i; q < j; ++q) {
                dog_result& R = results[idx[q]];
                std::vector<dog_blob>& v = res[q - i];
                R.raw_count = (int64_t)v.size();
                prune_blobs(v, P->sigma, P->prm.overlap);
                R.status = export_blobs(v, &R.blobs, &R.count);
            }
        }
        i = j;
        continue;
    chunk_fail:
        for (size_t q = i; q < j; ++q)
            results[idx[q]].status = rc;
        if (first_err == DOG_OK) {
            first_err = rc;
            first_msg = dog::last_error();
        }
        i = j;
    }
    if (first_err != DOG_OK)
        set_error(first_msg);
    return first_err;
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
    return dog_detect_device(c, static_cast<const float*>(c->input.p), height, width, width, &prm,
                             nullptr, blobs_out, count_out);
}

}  // extern "C"
