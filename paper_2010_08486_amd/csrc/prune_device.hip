// Overlap pruning and the radius histogram of a frame's blob list on the GPU
// (Sec. 4.1: overlapping blobs are pruned, or coalesced by averaging the
// radius, and the survivors' radii are histogrammed; the paper notes that
// these steps could move to the GPU as well).
//
// One workgroup per frame:
//   1. gather the frame's records from the candidate list into LDS (wave
//      ballot compaction), as 64-bit keys (y, x, scale, slot) that sort in
//      (y, x, scale) order, the response kept per slot;
//   2. bitonic sort of the keys in LDS;
//   3. every pair of blobs whose disks touch (centre distance below the sum
//      of the radii, with the starting sigmas) is listed per first blob, in
//      the order of the second, each with its overlap test already taken on
//      the starting sigmas; blobs are scanned in parallel, one per thread;
//   4. the pairs are visited in (y, x, scale) order exactly as the host
//      step does (a blob removed stops its own scan; of an overlapping pair
//      the smaller sigma goes, the later blob on a tie; coalescing gives the
//      survivor the mean sigma), re-taking the overlap test only where a
//      sigma has changed by coalescing: by one thread when coalescing, and
//      for plain pruning by one wave, which visits only the blobs with a
//      pair over the limit and takes their pairs 64 at a time.  Pairs whose disks do not touch have
//      overlap 0, which never exceeds the limit, and radii only shrink under
//      coalescing, so no other pair can ever overlap;
//   5. survivors are written in order with their final sigma, and counted in
//      the histogram bin of the ladder sigma nearest to their sigma (the
//      lower one on a tie; comparing sigmas is comparing radii sqrt(2) sigma).
// The overlap fraction is evaluated with the same FP64 operations, in the
// same order and without fused multiply-adds, as the host step.
#include <hip/hip_runtime.h>

#include "dog.h"
#include "dog_internal.h"
#include "prune_device.h"

namespace dog {

namespace {

constexpr int kNT = 256;   // threads per workgroup

// Key bit layout: y [33, 48), x [18, 33), scale [12, 18), slot [0, 12).
__device__ __forceinline__ uint64_t make_key(int y, int x, int scale, uint32_t slot)
{
    return ((uint64_t)(uint32_t)y << 33) | ((uint64_t)(uint32_t)x << 18) |
           ((uint64_t)(uint32_t)scale << 12) | (uint64_t)slot;
}
__device__ __forceinline__ int key_y(uint64_t k) { return (int)((k >> 33) & 0x7fff); }
__device__ __forceinline__ int key_x(uint64_t k) { return (int)((k >> 18) & 0x7fff); }
__device__ __forceinline__ int key_scale(uint64_t k) { return (int)((k >> 12) & 63); }
__device__ __forceinline__ uint32_t key_slot(uint64_t k) { return (uint32_t)(k & 4095); }

#pragma clang fp contract(off)

// Normalised overlap of two blobs (radius sqrt(2) sigma): area of the disks'
// intersection over the smaller disk's area.
__device__ double overlap_fraction(int y1, int x1, double s1, int y2, int x2, double s2)
{
    const double pi = 3.14159265358979323846;
    const double a = 1.4142135623730951 * s1, b = 1.4142135623730951 * s2;
    const double dy = (double)y1 - (double)y2, dx = (double)x1 - (double)x2;
    const double dist = sqrt(dy * dy + dx * dx);
    const double small = fmin(a, b);
    double area;
    if (dist >= a + b) {
        area = 0.0;
    } else if (dist <= fabs(a - b)) {
        area = pi * small * small;
    } else {
        const double d2 = dist * dist, a2 = a * a, b2 = b * b;
        const double ca = fmin(fmax((d2 + a2 - b2) / (2.0 * dist * a), -1.0), 1.0);
        const double cb = fmin(fmax((d2 + b2 - a2) / (2.0 * dist * b), -1.0), 1.0);
        const double kite = fmax(0.0, (-dist + a + b) * (dist + a - b) * (dist - a + b) * (dist + a + b));
        area = a2 * acos(ca) + b2 * acos(cb) - 0.5 * sqrt(kite);
    }
    return area / (pi * small * small);
}

// Disks that may touch: the host's quick test, whose margin keeps every pair
// the exact test could see as touching.
__device__ __forceinline__ bool may_touch(int ya, int xa, double sa, int yb, int xb, double sb)
{
    const double dy = (double)yb - (double)ya, dx = (double)xb - (double)xa;
    const double rs = 1.4142135623730951 * (sa + sb);
    return !(dy * dy + dx * dx > rs * rs * (1.0 + 1e-9));
}

#pragma clang fp contract(on)

// Exclusive prefix sum of v[0..n) in place, v[n] = total (n <= kNT * per).
__device__ void block_scan(uint32_t* v, uint32_t n, uint32_t* s_part)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (n + kNT - 1) / kNT;
    const uint32_t lo = tid * per, hi = min(n, lo + per);
    uint32_t sum = 0;
    for (uint32_t i = lo; i < hi; ++i)
        sum += v[i];
    s_part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int t = 0; t < kNT; ++t) {
            const uint32_t x = s_part[t];
            s_part[t] = run;
            run += x;
        }
        v[n] = run;
    }
    __syncthreads();
    uint32_t run = s_part[tid];
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t x = v[i];
        v[i] = run;
        run += x;
    }
    __syncthreads();
}

}  // namespace

__global__ void __launch_bounds__(kNT) k_prune(PruneArgs a)
{
    extern __shared__ __align__(16) char smem[];
    const uint32_t C = a.max_blobs;
    uint64_t* key = reinterpret_cast<uint64_t*>(smem);                 // C
    double* sg = reinterpret_cast<double*>(key + C);                    // C
    float* resp = reinterpret_cast<float*>(sg + C);                     // C
    uint32_t* off = reinterpret_cast<uint32_t*>(resp + C);              // C + 1
    uint16_t* pairs = reinterpret_cast<uint16_t*>(off + C + 1);         // max_pairs
    uint8_t* alive = reinterpret_cast<uint8_t*>(pairs + a.max_pairs);   // C

    __shared__ uint32_t s_n, s_out, s_status;
    __shared__ uint32_t s_part[kNT];
    __shared__ uint32_t s_wave[kNT / 64];
    __shared__ uint32_t s_hist[DOG_MAX_GAUSS];
    __shared__ double s_sig[DOG_MAX_GAUSS];   // the ladder's FP64 sigmas

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63, wv = tid >> 6;
    const int f = (int)blockIdx.x;
    PruneHead* head = reinterpret_cast<PruneHead*>(a.out + (uint64_t)f * a.out_stride);
    dog_blob* ob = reinterpret_cast<dog_blob*>(reinterpret_cast<char*>(head) + sizeof(PruneHead));
    if (tid == 0) {
        s_n = 0;
        s_out = 0;
        s_status = 0;
    }
    for (uint32_t i = tid; i < DOG_MAX_GAUSS; i += kNT) {
        s_hist[i] = 0;
        s_sig[i] = i < (uint32_t)a.k ? a.sig64[i] : 0.0;
    }
    __syncthreads();

    // ---- 1. gather this frame's records
    uint32_t n_all = a.n_direct;
    if (a.cand) {
        const uint32_t count = a.cand->count;
        if (count > a.cap) {
            if (tid == 0) {
                head->status = kPruneListOverflow;
                head->n_raw = count;
                head->n_out = 0;
            }
            return;
        }
        n_all = count;
    }
    for (uint32_t base = 0; base < n_all; base += kNT) {
        const uint32_t i = base + tid;
        bool mine = false;
        int y = 0, x = 0, s = 0;
        float r = 0.0f;
        if (i < n_all) {
            if (a.blob_in) {
                const dog_blob b = reinterpret_cast<const dog_blob*>(a.recs)[i];
                mine = true;
                y = b.y;
                x = b.x;
                s = b.scale;
                r = b.response;
            } else {
                const CandRec c = reinterpret_cast<const CandRec*>(a.recs)[i];
                mine = c.frame == f;
                y = c.y;
                x = c.x;
                s = c.scale;
                r = c.response;
            }
        }
        if (mine && (y < 0 || y > 32767 || x < 0 || x > 32767 || s < 0 || s >= a.k)) {
            s_status = 1;   // the key would not hold it
            mine = false;
        }
        const unsigned long long bal = __ballot(mine);
        uint32_t wbase = 0;
        if (lane == 0 && bal)
            wbase = atomicAdd(&s_n, (uint32_t)__popcll(bal));
        wbase = __shfl(wbase, 0);
        if (mine) {
            const uint32_t slot = wbase + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
            if (slot < C) {
                key[slot] = make_key(y, x, s, slot);
                resp[slot] = r;
            }
        }
    }
    __syncthreads();
    const uint32_t n = s_n;
    if (s_status) {
        if (tid == 0) {
            head->status = kPruneBadRecord;
            head->n_raw = n;
            head->n_out = 0;
        }
        return;
    }
    if (n > C) {
        if (tid == 0) {
            head->status = kPruneTooManyBlobs;
            head->n_raw = n;
            head->n_out = 0;
        }
        return;
    }

    // ---- 2. bitonic sort of the keys (padded to a power of two)
    uint32_t P = 1;
    while (P < n)
        P <<= 1;
    for (uint32_t i = n + tid; i < P; i += kNT)
        key[i] = ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = tid; t < P / 2; t += kNT) {
                const uint32_t i = 2 * t - (t & (stride - 1));
                const uint32_t j = i + stride;
                const bool up = (i & size) == 0;
                const uint64_t ki = key[i], kj = key[j];
                if ((ki > kj) == up) {
                    key[i] = kj;
                    key[j] = ki;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = tid; i < n; i += kNT) {
        sg[i] = s_sig[key_scale(key[i])];
        alive[i] = 1;
    }
    __syncthreads();

    // ---- 3. touching pairs, per first blob in the order of the second
    const bool prune = a.overlap < 1.0 && n >= 2;
    if (prune) {
        const double rmax = 1.4142135623730951 * a.sig_max;
        for (uint32_t i = tid; i < n; i += kNT) {
            const uint64_t ka = key[i];
            const int ya = key_y(ka), xa = key_x(ka);
            const double sa = sg[i];
            const double reach = 1.4142135623730951 * sa + rmax;
            uint32_t cnt = 0;
            for (uint32_t j = i + 1; j < n; ++j) {
                const uint64_t kb = key[j];
                if ((double)key_y(kb) - (double)ya >= reach)
                    break;
                cnt += may_touch(ya, xa, sa, key_y(kb), key_x(kb), sg[j]) ? 1u : 0u;
            }
            off[i] = cnt;
        }
        __syncthreads();
        block_scan(off, n, s_part);
        if (off[n] > a.max_pairs) {
            if (tid == 0) {
                head->status = kPruneTooManyPairs;
                head->n_raw = n;
                head->n_out = 0;
            }
            return;
        }
        for (uint32_t i = tid; i < n; i += kNT) {
            const uint64_t ka = key[i];
            const int ya = key_y(ka), xa = key_x(ka);
            const double sa = sg[i];
            const double reach = 1.4142135623730951 * sa + rmax;
            uint32_t o = off[i];
            bool any_over = false;
            for (uint32_t j = i + 1; j < n; ++j) {
                const uint64_t kb = key[j];
                const int yb = key_y(kb), xb = key_x(kb);
                if ((double)yb - (double)ya >= reach)
                    break;
                if (!may_touch(ya, xa, sa, yb, xb, sg[j]))
                    continue;
                const bool over = overlap_fraction(ya, xa, sa, yb, xb, sg[j]) > a.overlap;
                // bit 15: over the limit; bit 14: the first blob has the
                // smaller starting sigma (it goes, unless coalescing changes
                // a sigma first)
                pairs[o++] = (uint16_t)(j | (over ? 0x8000u : 0u) | (sa < sg[j] ? 0x4000u : 0u));
                any_over = any_over || over;
            }
            if (any_over)
                alive[i] = 3;   // bit 1: the blob has a pair over the limit
        }
        __syncthreads();

        // ---- 4. the greedy visits, in order
        if (!a.coalesce) {
            // Plain pruning: sigmas never change, so only the pairs over the
            // limit act, and which blob of such a pair goes is fixed.  Wave 0
            // visits the blobs that have such a pair, in order; a blob still
            // alive takes its pairs 64 at a time: of the pairs over the limit
            // whose second blob is alive, the second blobs before the first
            // pair the blob loses go, and the blob goes at that pair (its
            // scan stops), exactly as in the one-by-one visit.  Each second
            // blob appears once in a blob's pairs, so the lanes' updates do
            // not interact, and the wave's LDS accesses complete in order.
            if (wv == 0) {
                for (uint32_t base = 0; base < n; base += 64) {
                    const uint32_t il = base + lane;
                    unsigned long long todo = __ballot(il < n && (alive[il] & 2u));
                    while (todo) {
                        const uint32_t i = base + (uint32_t)__builtin_ctzll(todo);
                        todo &= todo - 1ull;
                        if (!(alive[i] & 1u))
                            continue;
                        const uint32_t e1 = off[i + 1];
                        for (uint32_t eb = off[i]; eb < e1; eb += 64) {
                            const uint32_t e = eb + lane;
                            bool act = false, lose = false;
                            uint32_t j = 0;
                            if (e < e1) {
                                const uint32_t w = pairs[e];
                                j = w & 0x0fffu;
                                act = (w & 0x8000u) && (alive[j] & 1u);
                                lose = act && (w & 0x4000u);
                            }
                            const unsigned long long lb = __ballot(lose);
                            const unsigned long long before = lb ? (lb & (0ull - lb)) - 1ull : ~0ull;
                            if (act && !lose && ((before >> lane) & 1ull))
                                alive[j] = (uint8_t)(alive[j] & 2u);
                            if (lb) {
                                if (lane == 0)
                                    alive[i] = (uint8_t)(alive[i] & 2u);
                                break;
                            }
                        }
                    }
                }
            }
        } else if (tid == 0) {
            // coalescing: a sigma may change at any pair, so one thread
            // visits every pair in order, re-taking the test where it has.
            // Only this loop writes sg, and sg[i] only in blob i's own scan,
            // so the blob's values stay in registers through its scan.
            for (uint32_t i = 0; i < n; ++i) {
                const uint32_t e0 = off[i], e1 = off[i + 1];
                if (e0 == e1 || !(alive[i] & 1u))
                    continue;
                const uint64_t ki = key[i];
                const int yi = key_y(ki), xi = key_x(ki);
                const double si0 = s_sig[key_scale(ki)];
                double si = sg[i];
                for (uint32_t e = e0; e < e1; ++e) {
                    const uint32_t w = pairs[e];
                    const uint32_t j = w & 0x0fffu;
                    if (!(alive[j] & 1u))
                        continue;
                    bool over = (w & 0x8000u) != 0;
                    const double sj = sg[j];
                    const uint64_t kj = key[j];
                    if (si != si0 || sj != s_sig[key_scale(kj)])
                        over = overlap_fraction(yi, xi, si, key_y(kj), key_x(kj), sj) > a.overlap;
                    if (!over)
                        continue;
                    const double mean = 0.5 * (si + sj);
                    if (si < sj) {
                        alive[i] = 0;
                        sg[j] = mean;
                        break;
                    }
                    alive[j] = 0;
                    si = mean;
                    sg[i] = mean;
                }
            }
        }
        __syncthreads();
    }

    // ---- 5. survivors in order, and their radius histogram
    for (uint32_t base = 0; base < n; base += kNT) {
        const uint32_t i = base + tid;
        const bool keep = i < n && (alive[i] & 1u);
        const unsigned long long bal = __ballot(keep);
        if (lane == 0)
            s_wave[wv] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t pos = s_out;
        for (uint32_t w = 0; w < wv; ++w)
            pos += s_wave[w];
        pos += (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (keep) {
            const uint64_t k = key[i];
            const int s = key_scale(k);
            dog_blob b;
            b.y = key_y(k);
            b.x = key_x(k);
            b.scale = s;
            b.sigma = (float)(a.coalesce ? sg[i] : s_sig[s]);
            b.response = resp[key_slot(k)];
            ob[pos] = b;
            // nearest ladder sigma to the output sigma, the lower on a tie
            const double v = (double)b.sigma;
            int bin = 0;
            while (bin < a.k && s_sig[bin] < v)
                ++bin;
            if (bin == a.k)
                bin = a.k - 1;
            else if (bin > 0 && v - s_sig[bin - 1] <= s_sig[bin] - v)
                bin -= 1;
            atomicAdd(&s_hist[bin], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t t = 0;
            for (uint32_t w = 0; w < kNT / 64; ++w)
                t += s_wave[w];
            s_out += t;
        }
        __syncthreads();
    }
    for (uint32_t i = tid; i < (uint32_t)a.k; i += kNT)
        head->hist[i] = s_hist[i];
    if (tid == 0) {
        head->status = kPruneDone;
        head->n_raw = n;
        head->n_out = s_out;
    }
}

}  // namespace dog

extern "C" {

size_t dogk_prune_lds_bytes(uint32_t max_blobs, uint32_t max_pairs)
{
    return (size_t)max_blobs * (8 + 8 + 4 + 4 + 1) + 4 + (size_t)max_pairs * 2;
}

hipError_t dogk_prune(const dog::PruneArgs* args, int n_frames, hipStream_t stream)
{
    const size_t lds = dogk_prune_lds_bytes(args->max_blobs, args->max_pairs);
    static size_t attr_set = 0;   // dynamic LDS the kernel has been allowed so far
    if (lds > attr_set) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&dog::k_prune),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess)
            return e;
        attr_set = lds;
    }
    void* params[] = {const_cast<dog::PruneArgs*>(args)};
    return hipLaunchKernel(reinterpret_cast<const void*>(&dog::k_prune), dim3(n_frames),
                           dim3(dog::kNT), params, lds, stream);
}

}  // extern "C"
