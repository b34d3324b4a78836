// Whole detector on a list of frames of any sizes: validation, grouping into
// launch sequences that fit the context's HBM budget, staging of host frames,
// the launch, and per-frame pruning.  Used by dog_detect_batch and the server.
#include <cstdlib>
#include <cstring>

#include "runtime.h"

namespace dog {

constexpr int kMaxSide = 32768;

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


// The frames of a batch chunk, already on the device, as consecutive groups
// of at most ctx->group_pixels pixels (at least one frame each) run on the
// context's lanes in turn: each lane is a child context with its own stream
// and workspace, so up to lane_count groups are in flight and a group's
// planes (about 72 bytes per pixel) stay near the Infinity Cache between its
// three kernels.  The lanes start after everything queued on s so far (the
// staged uploads), and every group is collected before the call returns.
// One group, a grouping of 0 pixels, or per-kernel timing run the chunk as
// one launch sequence on s instead.
// Results come back sorted and pruned, with each frame's count before
// pruning in raw[]; a group is pruned while the later groups run.
static int run_grouped(dog_context* ctx, const Plan& P, const std::vector<FrameIn>& fin,
                       hipStream_t s, std::vector<std::vector<dog_blob>>* res,
                       std::vector<int64_t>* raw)
{
    raw->assign(fin.size(), 0);
    auto finish = [&](size_t q) {
        (*raw)[q] = (int64_t)(*res)[q].size();
        prune_blobs((*res)[q], P.sigma, P.prm.overlap, P.prm.coalesce != 0);
    };
    const int64_t cap = ctx->group_pixels;
    std::vector<size_t> cut{0};
    int64_t px = 0;
    for (size_t q = 0; q < fin.size(); ++q) {
        const int64_t fpx = (int64_t)fin[q].H * fin[q].W;
        if (q > cut.back() && px + fpx > cap) {
            cut.push_back(q);
            px = 0;
        }
        px += fpx;
    }
    cut.push_back(fin.size());
    const size_t groups = cut.size() - 1;
    if (cap <= 0 || groups < 2 || ctx->lane_count < 2 || ctx->profiling) {
        const int rc = run_frames(ctx, P, fin, s, res, false, nullptr, nullptr, nullptr);
        if (rc == DOG_OK)
            for (size_t q = 0; q < fin.size(); ++q)
                finish(q);
        return rc;
    }

    const int K = std::min<int>(ctx->lane_count, (int)groups);
    while ((int)ctx->lanes.size() < K) {
        // lanes allocate out of this context's budget (ctx_alloc counts the
        // parent and every lane together)
        dog_context* l = nullptr;
        int rc = dog_context_create(ctx->device, ctx->budget, &l);
        if (rc != DOG_OK)
            return rc;
        l->parent = ctx;
        ctx->lanes.push_back(l);
    }
    if (!ctx->ev_fork)
        DOG_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    DOG_HIP(hipEventRecord(ctx->ev_fork, s));
    for (int k = 0; k < K; ++k) {
        dog_context* l = ctx->lanes[k];
        l->tuned = ctx->tuned;
        l->use_graphs = ctx->use_graphs;
        l->dct_min_taps = ctx->dct_min_taps;
        l->dct_forced = ctx->dct_forced;
        l->tuned_dct = ctx->tuned_dct;
        if (ctx->variant_forced) {
            int rc = ctx_set_variant(l, ctx->variant);
            if (rc != DOG_OK)
                return rc;
        }
        l->variant_forced = ctx->variant_forced;
        DOG_HIP(hipStreamWaitEvent(l->stream, ctx->ev_fork, 0));
    }
    res->assign(fin.size(), {});
    std::vector<size_t> lane_group(K, 0);
    int rc = DOG_OK;
    auto collect = [&](int k) {
        dog_context* l = ctx->lanes[k];
        if (!l->pending)
            return DOG_OK;
        std::vector<std::vector<dog_blob>> out;
        const int r = collect_frames(l, l->plan, &out);
        if (r != DOG_OK)
            return r;
        const size_t g = lane_group[k];
        for (size_t q = cut[g]; q < cut[g + 1]; ++q) {
            (*res)[q] = std::move(out[q - cut[g]]);
            finish(q);
        }
        return DOG_OK;
    };
    for (size_t g = 0; g < groups && rc == DOG_OK; ++g) {
        const int k = (int)(g % K);
        dog_context* l = ctx->lanes[k];
        if ((rc = collect(k)) != DOG_OK)
            break;
        const Plan* LP = nullptr;
        if ((rc = ctx_plan(l, &P.prm, &LP)) != DOG_OK)
            break;
        const std::vector<FrameIn> part(fin.begin() + cut[g], fin.begin() + cut[g + 1]);
        lane_group[k] = g;
        rc = launch_frames(l, *LP, part, l->stream, false, nullptr, nullptr, nullptr);
    }
    // every launch is collected, also after an error
    for (int k = 0; k < K; ++k) {
        const int r = collect(k);
        if (rc == DOG_OK)
            rc = r;
    }
    return rc;
}

int detect_frames(dog_context* ctx, const dog_params* params, int32_t n_frames,
                  const dog_frame* frames, hipStream_t s, dog_result* results)
{
    for (int32_t f = 0; f < n_frames; ++f)
        std::memset(&results[f], 0, sizeof(dog_result));
    int rc = DOG_OK;
    {
        hipError_t e = hipSetDevice(ctx->device);
        if (e != hipSuccess)
            return hip_fail(e, "hipSetDevice");
    }
    const Plan* P = nullptr;
    if ((rc = ctx_plan(ctx, params, &P)) != DOG_OK) {
        for (int32_t f = 0; f < n_frames; ++f)
            results[f].status = rc;
        return rc;
    }
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
                first_msg = last_error();
            }
            continue;
        }
        uint64_t b = frame_plane_bytes(*P, fr.height, fr.width);
        if (fr.on_device != 1)
            b += frame_input_bytes(fr.height, fr.width);
        idx.push_back(f);
        need.push_back(b);
    }
    // consecutive chunks that fit in what the budget leaves for planes and
    // inputs; the lanes' workspaces count against the same budget and are
    // released first when the next frame would not fit beside them
    auto room_now = [&]() -> uint64_t {
        const uint64_t fixed = ctx_total_used(ctx) - ctx->planes.bytes - ctx->input.bytes;
        return ctx->budget > fixed + ctx->room_margin ? ctx->budget - fixed - ctx->room_margin : 0;
    };
    uint64_t room = room_now();
    if (!idx.empty() && need[0] > room && !ctx->lanes.empty()) {
        for (dog_context* l : ctx->lanes)
            if ((rc = ctx_trim(l)) != DOG_OK)
                return rc;
        room = room_now();
    }
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
        // host frames: pageable ones through the pinned staging buffer (one
        // upload for all of them), pinned ones by DMA straight into place
        uint64_t in_bytes = 0, staged_bytes = 0;
        for (size_t q = i; q < j; ++q) {
            const dog_frame& fr = frames[idx[q]];
            const uint64_t b = ((uint64_t)fr.height * fr.width * sizeof(float) + 255) / 256 * 256;
            if (fr.on_device != 1)
                in_bytes += b;
            if (fr.on_device == 0)
                staged_bytes += b;
        }
        if (in_bytes) {
            if ((staged_bytes && (rc = ctx_pin(&ctx->h_input, staged_bytes)) != DOG_OK) ||
                (rc = ctx_alloc(ctx, &ctx->input, in_bytes, "input frames")) != DOG_OK)
                goto chunk_fail;
        }
        {
            std::vector<FrameIn> fin;
            uint64_t o = 0, so = 0;
            char* const dbase = static_cast<char*>(ctx->input.p);
            for (size_t q = i; q < j; ++q) {
                const dog_frame& fr = frames[idx[q]];
                const size_t row_bytes = (size_t)fr.width * sizeof(float);
                if (fr.on_device == 1) {
                    fin.push_back({fr.data, (int)fr.height, (int)fr.width, (long long)fr.row_stride});
                    continue;
                }
                if (fr.on_device == 2) {
                    hipError_t e = hipMemcpy2DAsync(dbase + o, row_bytes, fr.data,
                                                    (size_t)fr.row_stride * sizeof(float), row_bytes,
                                                    (size_t)fr.height, hipMemcpyHostToDevice, s);
                    if (e != hipSuccess) {
                        rc = hip_fail(e, "hipMemcpy2DAsync(pinned input)");
                        goto chunk_fail;
                    }
                } else {
                    char* hp = static_cast<char*>(ctx->h_input.p) + so;
                    for (int64_t y = 0; y < fr.height; ++y)
                        std::memcpy(hp + (size_t)y * row_bytes, fr.data + y * fr.row_stride, row_bytes);
                    so += ((uint64_t)fr.height * row_bytes + 255) / 256 * 256;
                }
                fin.push_back({reinterpret_cast<const float*>(dbase + o), (int)fr.height,
                               (int)fr.width, (long long)fr.width});
                o += ((uint64_t)fr.height * row_bytes + 255) / 256 * 256;
            }
            // staged frames keep their order in the input area, where pinned
            // frames may sit between them: one upload per run of staged frames
            if (staged_bytes) {
                uint64_t d = 0, h = 0, run_d = 0, run_h = 0, run_b = 0;
                for (size_t q = i; q <= j; ++q) {
                    const bool end = q == j;
                    const dog_frame* fr = end ? nullptr : &frames[idx[q]];
                    if (!end && fr->on_device == 1)
                        continue;
                    if ((end || fr->on_device == 2) && run_b) {
                        hipError_t e = hipMemcpyAsync(dbase + run_d,
                                                      static_cast<char*>(ctx->h_input.p) + run_h, run_b,
                                                      hipMemcpyHostToDevice, s);
                        if (e != hipSuccess) {
                            rc = hip_fail(e, "hipMemcpyAsync(input)");
                            goto chunk_fail;
                        }
                        run_b = 0;
                    }
                    if (end)
                        break;
                    const uint64_t b = ((uint64_t)fr->height * fr->width * sizeof(float) + 255) / 256 * 256;
                    if (fr->on_device == 0) {
                        if (run_b == 0) {
                            run_d = d;
                            run_h = h;
                        }
                        run_b += b;
                        h += b;
                    }
                    d += b;
                }
            }
            std::vector<std::vector<dog_blob>> res;
            std::vector<int64_t> raw;
            rc = run_grouped(ctx, *P, fin, s, &res, &raw);
            if (rc != DOG_OK)
                goto chunk_fail;
            for (size_t q = i; q < j; ++q) {
                dog_result& R = results[idx[q]];
                R.raw_count = raw[q - i];
                R.status = export_blobs(res[q - i], &R.blobs, &R.count);
            }
        }
        i = j;
        continue;
    chunk_fail:
        for (size_t q = i; q < j; ++q)
            results[idx[q]].status = rc;
        if (first_err == DOG_OK) {
            first_err = rc;
            first_msg = last_error();
        }
        i = j;
    }
    if (first_err != DOG_OK)
        set_error(first_msg);
    return first_err;
}


}  // namespace dog
