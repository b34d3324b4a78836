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
        const uint64_t pitch = ((uint64_t)fr.height + 63) / 64 * 64;
        uint64_t b = 2ull * P->n_g * (uint64_t)fr.width * pitch * sizeof(float) + 256;
        if (fr.on_device != 1)
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
            rc = run_frames(ctx, *P, fin, s, &res, false, nullptr, nullptr, nullptr);
            if (rc != DOG_OK)
                goto chunk_fail;
            for (size_t q = i; q < j; ++q) {
                dog_result& R = results[idx[q]];
                std::vector<dog_blob>& v = res[q - i];
                R.raw_count = (int64_t)v.size();
                prune_blobs(v, P->sigma, P->prm.overlap, P->prm.coalesce != 0);
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
            first_msg = last_error();
        }
        i = j;
    }
    if (first_err != DOG_OK)
        set_error(first_msg);
    return first_err;
}


}  // namespace dog
