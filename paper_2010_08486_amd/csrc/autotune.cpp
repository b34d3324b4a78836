// Autotuner: for a frame shape and ladder, time the kernel variants (tile
// geometry S / R / waves, local-maximum rows) and, on frames whose sides are
// powers of two, the transform threshold (how many of the widest planes are
// blurred in the cosine-transform domain) on a representative device frame
// with the library's own per-kernel event timing, and keep the fastest.
// Choices are kept per (shape, radii) in the context and can be saved to and
// loaded from a JSON cache keyed by architecture and kernel source, so a
// production process starts tuned.  Every variant computes bitwise identical
// results (taps are summed in the same order); the transform threshold
// changes the planes it moves to the transform domain within the plane
// tolerance, and is applied per frame by its own shape, so a frame gives the
// same result alone and in any batch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <sstream>

#include "runtime.h"

#ifndef DOG_KERNEL_HASH
#define DOG_KERNEL_HASH "unknown"
#endif

namespace dog {

static std::string radii_sig(const Plan& P)
{
    std::string s;
    for (size_t i = 0; i < P.r.size(); ++i) {
        if (i)
            s += ',';
        s += std::to_string(P.r[i]);
    }
    return s;
}

static std::string shape_key(int64_t H, int64_t W, const Plan& P)
{
    return std::to_string(H) + "x" + std::to_string(W) + "|" + radii_sig(P);
}

// Variant for a launch over `frames`: the pinned one, else the tuned choice
// of the shape holding the most pixels, else that of the tuned shape with the
// same radii nearest in pixel count, else the built-in default.
int choose_variant(const dog_context* c, const std::vector<FrameIn>& frames, const Plan& P)
{
    if (c->variant_forced)
        return c->variant;
    if (c->tuned.empty() || frames.empty())
        return c->variant_auto;
    std::vector<std::pair<std::pair<int, int>, double>> px;
    for (const FrameIn& f : frames) {
        bool found = false;
        for (auto& e : px)
            if (e.first.first == f.H && e.first.second == f.W) {
                e.second += (double)f.H * f.W;
                found = true;
            }
        if (!found)
            px.push_back({{f.H, f.W}, (double)f.H * f.W});
    }
    auto best = std::max_element(px.begin(), px.end(),
                                 [](const auto& a, const auto& b) { return a.second < b.second; });
    const int H = best->first.first, W = best->first.second;
    auto it = c->tuned.find(shape_key(H, W, P));
    if (it != c->tuned.end())
        return it->second;
    const std::string sig = "|" + radii_sig(P);
    double best_d = 1e300;
    int v = c->variant_auto;
    for (const auto& kv : c->tuned) {
        const std::string& k = kv.first;
        if (k.size() < sig.size() || k.compare(k.size() - sig.size(), sig.size(), sig) != 0)
            continue;
        long long h = 0, w = 0;
        if (std::sscanf(k.c_str(), "%lldx%lld|", &h, &w) != 2)
            continue;
        const double d = std::fabs(std::log((double)h * w) - std::log((double)H * W));
        if (d < best_d) {
            best_d = d;
            v = kv.second;
        }
    }
    return v;
}

int frame_min_taps(const dog_context* c, int H, int W, const Plan& P)
{
    if (c->dct_forced)
        return c->dct_min_taps;
    if (c->tuned_dct.empty())
        return 0;
    const auto it = c->tuned_dct.find(shape_key(H, W, P));
    return it == c->tuned_dct.end() ? 0 : it->second;
}

}  // namespace dog

using namespace dog;

extern "C" {

int dog_autotune(dog_context* ctx, const dog_params* params, const float* d_image, int64_t height,
                 int64_t width, int64_t row_stride, int32_t reps, int32_t* variant_out,
                 double* us_out)
{
    if (!ctx || !params || !d_image || reps < 0) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    int rc = check_image(d_image, height, width, row_stride);
    if (rc != DOG_OK)
        return rc;
    if (ctx->pending) {
        set_error("a launch of dog_detect_device_async has not been finished");
        return DOG_EBUSY;
    }
    DOG_HIP(hipSetDevice(ctx->device));
    const Plan* P = nullptr;
    if ((rc = ctx_plan(ctx, params, &P)) != DOG_OK)
        return rc;
    const Plan plan = *P;
    if (reps == 0)
        reps = 5;
    const float* img = d_image;
    const std::vector<FrameIn> fr{{img, (int)height, (int)width, (long long)row_stride}};
    const int saved_variant = ctx->variant;
    const bool saved_forced = ctx->variant_forced;
    const bool saved_prof = ctx->profiling;
    const bool saved_dct_forced = ctx->dct_forced;
    const int saved_dct = ctx->dct_min_taps;
    ctx->variant_forced = true;
    ctx->profiling = true;
    ctx->dct_forced = true;
    std::vector<std::vector<dog_blob>> out;
    // median over reps of the kernel microseconds of one frame with variant v
    // and threshold mt (a median, so one slow launch cannot flip a choice)
    auto time_it = [&](int v, int mt, double* us) -> int {
        int r = ctx_set_variant(ctx, v);
        if (r != DOG_OK)
            return r;
        ctx->dct_min_taps = mt;
        // one untimed launch (tables, first touch), then reps timed ones
        if ((r = run_frames(ctx, plan, fr, ctx->stream, &out, false, nullptr, nullptr, nullptr)) !=
            DOG_OK)
            return r;
        std::vector<double> per;
        for (int i = 0; i < reps; ++i) {
            for (double& m : ctx->kernel_ms)
                m = 0.0;
            ctx->kernel_launches = 0;
            if ((r = run_frames(ctx, plan, fr, ctx->stream, &out, false, nullptr, nullptr,
                                nullptr)) != DOG_OK)
                return r;
            double ms = 0.0;
            for (double m : ctx->kernel_ms)
                ms += m;
            per.push_back(ms * 1e3 / (double)std::max<int64_t>(1, ctx->kernel_launches));
        }
        std::sort(per.begin(), per.end());
        const size_t n = per.size();
        *us = n % 2 ? per[n / 2] : 0.5 * (per[n / 2 - 1] + per[n / 2]);
        return DOG_OK;
    };
    // every variant at a threshold; the built-in default stands unless
    // another variant beats it by more than the timing noise (2 %), so
    // repeated tuning gives the same choice
    std::vector<double> times(dogk_num_variants(), 1e300);
    auto best_variant = [&](int mt, int* best) -> int {
        double best_us = 1e300;
        *best = -1;
        for (int v = 0; v < dogk_num_variants(); ++v) {
            const int r = time_it(v, mt, &times[v]);
            if (r != DOG_OK)
                return r;
            if (times[v] < best_us) {
                best_us = times[v];
                *best = v;
            }
        }
        if (*best != ctx->variant_auto && times[ctx->variant_auto] <= best_us * 1.02)
            *best = ctx->variant_auto;
        return DOG_OK;
    };
    int best = -1, best_mt = 0;
    rc = best_variant(0, &best);
    if (rc == DOG_OK && frame_dct_ok((int)height, (int)width)) {
        // thresholds: none, then the widest plane, the two widest, ...
        std::vector<int> cand;
        for (int p = plan.n_g - 1; p >= 0; --p) {
            const int taps = 2 * plan.r[p] + 1;
            if (cand.empty() || cand.back() != taps)
                cand.push_back(taps);
        }
        double us0 = times[best], best_us = us0;
        for (int mt : cand) {
            double us = 0.0;
            if ((rc = time_it(best, mt, &us)) != DOG_OK)
                break;
            if (us < best_us) {
                best_us = us;
                best_mt = mt;
            }
        }
        // the direct blur (bitwise the same for every variant) stands
        // unless the transform domain is clearly faster
        if (rc == DOG_OK && best_mt > 0 && us0 <= best_us * 1.02)
            best_mt = 0;
        if (rc == DOG_OK && best_mt > 0)
            rc = best_variant(best_mt, &best);   // the geometry for the planes left direct
    }
    ctx->profiling = saved_prof;
    ctx->variant_forced = saved_forced;
    ctx->dct_forced = saved_dct_forced;
    ctx->dct_min_taps = saved_dct;
    for (double& m : ctx->kernel_ms)
        m = 0.0;
    ctx->kernel_launches = 0;
    drop_graph(ctx);
    const int rc2 = ctx_set_variant(ctx, saved_variant);
    if (rc != DOG_OK)
        return rc;
    if (rc2 != DOG_OK)
        return rc2;
    if (us_out)
        for (int v = 0; v < dogk_num_variants(); ++v)
            us_out[v] = times[v];
    ctx->tuned[shape_key(height, width, plan)] = best;
    ctx->tuned_dct[shape_key(height, width, plan)] = best_mt;
    if (variant_out)
        *variant_out = best;
    return DOG_OK;
}

int dog_autotune_save(dog_context* ctx, const char* path)
{
    if (!ctx || !path) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    FILE* fp = std::fopen(path, "w");
    if (!fp) {
        set_error(std::string("cannot write ") + path);
        return DOG_EINVAL;
    }
    std::fprintf(fp, "{\n  \"arch\": \"gfx950\",\n  \"kernels\": \"%s\",\n  \"entries\": [\n",
                 DOG_KERNEL_HASH);
    size_t i = 0;
    for (const auto& kv : ctx->tuned) {
        const std::string& k = kv.first;
        const size_t bar = k.find('|');
        const auto d = ctx->tuned_dct.find(k);
        std::fprintf(fp,
                     "    {\"shape\": \"%s\", \"radii\": \"%s\", \"variant\": %d, "
                     "\"min_taps\": %d}%s\n",
                     k.substr(0, bar).c_str(), k.substr(bar + 1).c_str(), kv.second,
                     d == ctx->tuned_dct.end() ? 0 : d->second,
                     ++i < ctx->tuned.size() ? "," : "");
    }
    std::fprintf(fp, "  ]\n}\n");
    std::fclose(fp);
    return DOG_OK;
}

// Reads the format written above; entries of another architecture or kernel
// source are ignored (returns DOG_OK with nothing loaded).
int dog_autotune_load(dog_context* ctx, const char* path)
{
    if (!ctx || !path) {
        set_error("invalid argument");
        return DOG_EINVAL;
    }
    FILE* fp = std::fopen(path, "r");
    if (!fp) {
        set_error(std::string("cannot read ") + path);
        return DOG_EINVAL;
    }
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), fp)) > 0)
        text.append(buf, got);
    std::fclose(fp);
    const std::string want_k = std::string("\"kernels\": \"") + DOG_KERNEL_HASH + "\"";
    if (text.find("\"arch\": \"gfx950\"") == std::string::npos ||
        text.find(want_k) == std::string::npos)
        return DOG_OK;
    std::istringstream in(text);
    std::string line;
    const int nv = dogk_num_variants();
    while (std::getline(in, line)) {
        char shape[64], radii[1024];
        int v = -1, mt = 0;
        const size_t p = line.find("{\"shape\"");
        if (p == std::string::npos)
            continue;
        const int got = std::sscanf(
            line.c_str() + p,
            "{\"shape\": \"%63[^\"]\", \"radii\": \"%1023[^\"]\", \"variant\": %d, \"min_taps\": %d",
            shape, radii, &v, &mt);
        if (got >= 3 && v >= 0 && v < nv && mt >= 0) {
            const std::string key = std::string(shape) + "|" + radii;
            ctx->tuned[key] = v;
            ctx->tuned_dct[key] = got == 4 ? mt : 0;
        }
    }
    return DOG_OK;
}

int dog_autotune_transform(dog_context* ctx, const dog_params* params, int64_t height,
                           int64_t width, int32_t* min_taps_out)
{
    if (!ctx || !params || !min_taps_out) {
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
    *min_taps_out = frame_dct_ok((int)height, (int)width)
                        ? frame_min_taps(ctx, (int)height, (int)width, P)
                        : 0;
    return DOG_OK;
}

int dog_autotune_choice(dog_context* ctx, const dog_params* params, int64_t height, int64_t width,
                        int32_t* variant_out)
{
    if (!ctx || !params || !variant_out) {
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
    const std::vector<FrameIn> fr{{nullptr, (int)height, (int)width, (long long)width}};
    const bool forced = ctx->variant_forced;
    ctx->variant_forced = false;
    *variant_out = choose_variant(ctx, fr, P);
    ctx->variant_forced = forced;
    return DOG_OK;
}

}  // extern "C"
