// Preprocessing of a frame before detection (Sec. 4.1, optional first step):
// Gaussian smoothing, then a contrast stretch to [0, 1] that saturates a
// given fraction of the pixels, half at each end.
//
//   S = G(sigma) * I          truncated at radius floor(4 sigma + 0.5),
//                             normalised weights, half-sample reflection
//   lo, hi = the m-th smallest and m-th largest value of S,
//            m = floor(saturated * N / 2)   (exact order statistics)
//   out = clamp((S - lo) / (hi - lo), 0, 1), or 0 where hi == lo
//
// Smoothing: one workgroup per 64 x 32 output tile; the input tile with its
// halo is staged in LDS, blurred along rows into a second LDS tile, then
// along columns into the output (taps in ascending order, fp32 FMAs).
// Order statistics: an exact radix select on the order-preserving integer
// keys of the fp32 values, over digits of 11, 11 and 10 bits.  The smoothing
// kernel histograms the top digit of its outputs; each later kernel first
// finds, in every workgroup, the digits already fixed (a scan of the
// previous histograms), then histograms the next digit of the keys under
// them; the last one finds the limits and applies the stretch.  Four
// launches, all on the stream, each clearing a histogram that the next
// call needs zero; the host reads nothing unless it asks for the limits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace dogpre {

constexpr int kTX = 64;        // output columns per smoothing tile
constexpr int kTY = 32;        // output rows per smoothing tile
constexpr int kMaxR = 16;      // largest smoothing radius (sigma <= 3.9 at truncate 4)
constexpr int kBins = 2048;    // digit histogram bins (11 bits)
constexpr int kBatch = 8;      // keys loaded per thread before counting

// State of the select, in device memory (the limits sit at byte 16): the
// limits, then for passes 0 and 1 each target's fixed key bits so far and
// its rank among the keys that share them, written by workgroup 0 of the
// next kernel and read by the kernel after it.
struct SelectState {
    uint32_t pad0_[4];
    float limit[2];
    uint32_t pad1_[2];
    uint32_t prefix[2][2];
    uint32_t rank[2][2];
};

// Scratch layout: state, then the digit histograms of the three passes:
// pass 0 (top 11 bits, one histogram: both targets see every key), pass 1
// (next 11 bits, one per target), pass 2 (low 10 bits, one per target).
constexpr size_t kOffH0 = 256;
constexpr size_t kOffH1 = kOffH0 + kBins * 4;
constexpr size_t kOffH2 = kOffH1 + 2 * kBins * 4;
constexpr size_t kScratch = kOffH2 + 2 * 1024 * 4;

__device__ __forceinline__ int reflect(int t, int n)
{
    if ((unsigned)t < (unsigned)n)
        return t;
    const int p = 2 * n;
    int u = t % p;
    if (u < 0)
        u += p;
    return u < n ? u : p - 1 - u;
}

// Order-preserving map of finite floats to unsigned integers and back.
__device__ __forceinline__ uint32_t key_of(float f)
{
    const uint32_t b = __builtin_bit_cast(uint32_t, f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float value_of(uint32_t k)
{
    const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __builtin_bit_cast(float, b);
}

// h[d] += 1 for every lane with `take`: the lanes sharing the first active
// lane's digit add together with one LDS atomic (the smoothed values of a
// frame crowd into a few digits, where per-lane atomics on one address
// would serialise), the others add one by one.  Called by all lanes of the
// wave together.
__device__ __forceinline__ void wave_hist_add(uint32_t* h, uint32_t d, bool take)
{
    const unsigned long long act = __ballot(take);
    if (!act)
        return;
    const int leader = __builtin_ctzll(act);
    const uint32_t dl = (uint32_t)__builtin_amdgcn_readlane((int)d, leader);
    const unsigned long long grp = __ballot(take && d == dl);
    if ((int)(threadIdx.x & 63) == leader)
        atomicAdd(&h[dl], (uint32_t)__popcll(grp));
    else if (take && d != dl)
        atomicAdd(&h[d], 1u);
}

// Run by the first wave of a workgroup: the digit whose bin holds the
// rank-th smallest key (0-based) of an nb-bin histogram (nb = 1024 or 2048)
// and the rank within that bin, both returned to every lane of the wave.
__device__ void wave_pick(const uint32_t* hist, int nb, uint32_t rank, uint32_t* digit,
                          uint32_t* rem)
{
    const int lane = threadIdx.x & 63;
    const int per = nb / 64;   // 16 or 32 bins per lane
    uint32_t c[32];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        c[i] = i < per ? hist[lane * per + i] : 0u;
        sum += c[i];
    }
    // inclusive scan over the lanes
    uint32_t inc = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)inc, off);
        if (lane >= off)
            inc += v;
    }
    const uint32_t before = inc - sum;
    const bool here = rank >= before && rank < inc;
    uint32_t dg = 0, rm = 0;
    if (here) {
        uint32_t acc = before;
        bool found = false;
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            if (!found && i < per && rank < acc + c[i]) {
                dg = (uint32_t)(lane * per + i);
                rm = rank - acc;
                found = true;
            }
            acc += c[i];
        }
    }
    const unsigned long long who = __ballot(here);
    const int src = who ? __builtin_ctzll(who) : 0;
    *digit = (uint32_t)__builtin_amdgcn_readlane((int)dg, src);
    *rem = (uint32_t)__builtin_amdgcn_readlane((int)rm, src);
}

// Smoothing of one 64 x 32 tile (r = 0 with the single weight 1 copies),
// and the pass-0 digit histogram of the smoothed values.
__global__ void __launch_bounds__(256) k_smooth(const float* __restrict__ in, int H, int W,
                                                long long stride, const float* __restrict__ w,
                                                int r, float* __restrict__ out,
                                                uint32_t* __restrict__ hist0,
                                                uint32_t* __restrict__ hist1)
{
    __shared__ float tile[(kTY + 2 * kMaxR) * (kTX + 2 * kMaxR)];
    __shared__ float rows[(kTY + 2 * kMaxR) * kTX];
    __shared__ uint32_t h[kBins];
    const int tx0 = blockIdx.x * kTX, ty0 = blockIdx.y * kTY;
    const int TW = kTX + 2 * r, TH = kTY + 2 * r;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x)
        h[i] = 0u;
    // the pass-1 histograms must be zero before the next kernel counts
    const int wg = blockIdx.y * gridDim.x + blockIdx.x;
    for (int i = wg * blockDim.x + threadIdx.x; i < 2 * kBins; i += gridDim.x * gridDim.y * blockDim.x)
        hist1[i] = 0u;
    // the input tile with its halo, eight loads in flight per thread
    for (int i0 = 0; i0 < TW * TH; i0 += 8 * 256) {
        float v[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int i = i0 + b * 256 + threadIdx.x;
            v[b] = 0.0f;
            if (i < TW * TH) {
                const int yy = i / TW, xx = i - yy * TW;
                const int y = reflect(ty0 - r + yy, H), x = reflect(tx0 - r + xx, W);
                v[b] = in[(long long)y * stride + x];
            }
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int i = i0 + b * 256 + threadIdx.x;
            if (i < TW * TH)
                tile[i] = v[b];
        }
    }
    __syncthreads();
    // along rows: rows[yy][x] = sum_j w[j] tile[yy][x + j]
    for (int i = threadIdx.x; i < TH * kTX; i += blockDim.x) {
        const int yy = i / kTX, x = i - yy * kTX;
        const float* t = tile + yy * TW + x;
        float acc = 0.0f;
        for (int j = 0; j <= 2 * r; ++j)
            acc = __builtin_fmaf(w[j], t[j], acc);
        rows[yy * kTX + x] = acc;
    }
    __syncthreads();
    // along columns, into the output (kTY * kTX / 256 = 8 uniform rounds)
    for (int i = threadIdx.x; i < kTY * kTX; i += blockDim.x) {
        const int y = i / kTX, x = i - y * kTX;
        const float* t = rows + y * kTX + x;
        float acc = 0.0f;
        for (int j = 0; j <= 2 * r; ++j)
            acc = __builtin_fmaf(w[j], t[j * kTX], acc);
        const bool valid = ty0 + y < H && tx0 + x < W;
        if (valid)
            out[(long long)(ty0 + y) * W + tx0 + x] = acc;
        wave_hist_add(h, key_of(acc) >> 21, valid);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += blockDim.x)
        if (h[i])
            atomicAdd(&hist0[i], h[i]);
}

// Each target's next digit from `hist` (one nb-bin histogram per target,
// or one shared when `shared`): the workgroup copies the histograms into
// LDS (`stage`, 2 nb words) with coalesced loads, the first wave picks, and
// the results reach every thread through LDS.
__device__ void pick_both(const uint32_t* __restrict__ hist, int nb, bool shared,
                          const uint32_t rank[2], uint32_t* stage, uint32_t* s_res,
                          uint32_t digit[2], uint32_t rem[2])
{
    const int words = shared ? nb : 2 * nb;
    for (int i = 4 * threadIdx.x; i < words; i += 4 * blockDim.x)
        *reinterpret_cast<uint4*>(stage + i) = *reinterpret_cast<const uint4*>(hist + i);
    __syncthreads();
    if (threadIdx.x < 64) {
        for (int tg = 0; tg < 2; ++tg) {
            uint32_t dg, rm;
            wave_pick(stage + (shared ? 0 : tg * nb), nb, rank[tg], &dg, &rm);
            if (threadIdx.x == 0) {
                s_res[2 * tg] = dg;
                s_res[2 * tg + 1] = rm;
            }
        }
    }
    __syncthreads();
    for (int tg = 0; tg < 2; ++tg) {
        digit[tg] = s_res[2 * tg];
        rem[tg] = s_res[2 * tg + 1];
    }
}

// Pass 1: both targets' top digit from hist0, then the histograms of the
// next 11 bits of the keys under each.
__global__ void __launch_bounds__(256) k_select_pass1(const float* __restrict__ s, long long n,
                                                      const uint32_t* __restrict__ hist0,
                                                      uint32_t* __restrict__ hist1,
                                                      uint32_t* __restrict__ hist2,
                                                      uint32_t rank_lo, uint32_t rank_hi,
                                                      SelectState* st)
{
    __shared__ __align__(16) uint32_t h[2 * kBins];
    __shared__ uint32_t s_res[4];
    const uint32_t rk0[2] = {rank_lo, rank_hi};
    uint32_t d0[2], rk[2];
    pick_both(hist0, kBins, true, rk0, h, s_res, d0, rk);
    for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x)
        h[i] = 0u;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x < 2) {
        st->prefix[0][threadIdx.x] = d0[threadIdx.x];
        st->rank[0][threadIdx.x] = rk[threadIdx.x];
    }
    // the pass-2 histograms must be zero before the next kernel counts
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * 1024; i += gridDim.x * blockDim.x)
        hist2[i] = 0u;
    const long long step = (long long)gridDim.x * blockDim.x * kBatch;
    for (long long base = (long long)blockIdx.x * blockDim.x * kBatch; base < n; base += step) {
        uint32_t k[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const long long i = base + b * blockDim.x + threadIdx.x;
            k[b] = i < n ? key_of(s[i]) : 0u;
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const bool valid = base + b * blockDim.x + threadIdx.x < n;
            const uint32_t d = (k[b] >> 10) & 0x7ffu;
            wave_hist_add(h, d, valid && (k[b] >> 21) == d0[0]);
            wave_hist_add(h + kBins, d, valid && (k[b] >> 21) == d0[1]);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x)
        if (h[i])
            atomicAdd(&hist1[i], h[i]);
}

// Pass 2: the second digits from hist1, then the histograms of the low 10
// bits of the keys that share each target's top 22 bits.
__global__ void __launch_bounds__(256) k_select_pass2(const float* __restrict__ s, long long n,
                                                      const uint32_t* __restrict__ hist1,
                                                      uint32_t* __restrict__ hist2,
                                                      SelectState* st)
{
    __shared__ __align__(16) uint32_t stage[2 * kBins];
    __shared__ uint32_t s_res[4];
    uint32_t* h = stage;   // the pass-2 histograms reuse the staging area
    const uint32_t d0[2] = {st->prefix[0][0], st->prefix[0][1]};
    const uint32_t rk0[2] = {st->rank[0][0], st->rank[0][1]};
    uint32_t d1[2], rk[2], pre[2];
    pick_both(hist1, kBins, false, rk0, stage, s_res, d1, rk);
    for (int i = threadIdx.x; i < 2 * 1024; i += blockDim.x)
        h[i] = 0u;
    __syncthreads();
    for (int tg = 0; tg < 2; ++tg)
        pre[tg] = (d0[tg] << 11) | d1[tg];
    if (blockIdx.x == 0 && threadIdx.x < 2) {
        st->prefix[1][threadIdx.x] = pre[threadIdx.x];
        st->rank[1][threadIdx.x] = rk[threadIdx.x];
    }
    const long long step = (long long)gridDim.x * blockDim.x * kBatch;
    for (long long base = (long long)blockIdx.x * blockDim.x * kBatch; base < n; base += step) {
        uint32_t k[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const long long i = base + b * blockDim.x + threadIdx.x;
            k[b] = i < n ? key_of(s[i]) : 0u;
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const bool valid = base + b * blockDim.x + threadIdx.x < n;
            const uint32_t d = k[b] & 0x3ffu;
            wave_hist_add(h, d, valid && (k[b] >> 10) == pre[0]);
            wave_hist_add(h + 1024, d, valid && (k[b] >> 10) == pre[1]);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * 1024; i += blockDim.x)
        if (h[i])
            atomicAdd(&hist2[i], h[i]);
}

// The last digits from hist2 give the limits (workgroup 0 stores them for
// the host), then the stretch.
__global__ void __launch_bounds__(256) k_stretch(const float* __restrict__ s, long long n,
                                                 uint32_t* __restrict__ hist0,
                                                 const uint32_t* __restrict__ hist2,
                                                 SelectState* st, float* __restrict__ out)
{
    __shared__ __align__(16) uint32_t stage[2 * 1024];
    __shared__ uint32_t s_res[4];
    const uint32_t pre[2] = {st->prefix[1][0], st->prefix[1][1]};
    const uint32_t rk1[2] = {st->rank[1][0], st->rank[1][1]};
    uint32_t d2[2], rk[2];
    pick_both(hist2, 1024, false, rk1, stage, s_res, d2, rk);
    const float lo = value_of((pre[0] << 10) | d2[0]);
    const float hi = value_of((pre[1] << 10) | d2[1]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->limit[0] = lo;
        st->limit[1] = hi;
    }
    // leave the pass-0 histogram zero for the next call's smoothing kernel
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kBins; i += gridDim.x * blockDim.x)
        hist0[i] = 0u;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        float v = 0.0f;
        if (hi > lo)
            v = fminf(fmaxf((s[i] - lo) / (hi - lo), 0.0f), 1.0f);
        out[i] = v;
    }
}

}  // namespace dogpre

extern "C" {

// Scratch the launcher needs in device memory: select state + histograms.
size_t dogk_preprocess_scratch_bytes() { return dogpre::kScratch; }

int dogk_preprocess_max_radius() { return dogpre::kMaxR; }

// Queue the preprocessing of one frame on `stream`.  d_w: 2r+1 fp32 weights
// on the device (r = 0 with the weight 1: no smoothing); d_s: H x W dense
// smoothed image (may equal d_out, then the stretch runs in place);
// d_scratch: at least dogk_preprocess_scratch_bytes(), 256-byte aligned,
// whose histograms are zero before the first call (each call leaves them
// zero for the next).
// rank_lo/rank_hi: the 0-based ranks of the limits.  The two limits
// (floats) sit at d_scratch + 16 once the stream has passed the launch.
hipError_t dogk_preprocess(const float* d_in, int H, int W, long long stride, const float* d_w,
                           int r, float* d_s, float* d_out, void* d_scratch, uint32_t rank_lo,
                           uint32_t rank_hi, hipStream_t stream)
{
    using namespace dogpre;
    const long long n = (long long)H * W;
    char* base = static_cast<char*>(d_scratch);
    SelectState* st = reinterpret_cast<SelectState*>(base);
    uint32_t* h0 = reinterpret_cast<uint32_t*>(base + kOffH0);
    uint32_t* h1 = reinterpret_cast<uint32_t*>(base + kOffH1);
    uint32_t* h2 = reinterpret_cast<uint32_t*>(base + kOffH2);
    const dim3 grid((unsigned)((W + kTX - 1) / kTX), (unsigned)((H + kTY - 1) / kTY));
    hipLaunchKernelGGL(k_smooth, grid, dim3(256), 0, stream, d_in, H, W, stride, d_w, r, d_s, h0, h1);
    const long long g = std::max<long long>(1, std::min<long long>((n + 2047) / 2048, 4096));
    hipLaunchKernelGGL(k_select_pass1, dim3((unsigned)g), dim3(256), 0, stream, (const float*)d_s,
                       n, (const uint32_t*)h0, h1, h2, rank_lo, rank_hi, st);
    hipLaunchKernelGGL(k_select_pass2, dim3((unsigned)g), dim3(256), 0, stream, (const float*)d_s,
                       n, (const uint32_t*)h1, h2, st);
    const long long gs = std::max<long long>(1, std::min<long long>((n + 1023) / 1024, 4096));
    hipLaunchKernelGGL(k_stretch, dim3((unsigned)gs), dim3(256), 0, stream, (const float*)d_s, n, h0,
                       (const uint32_t*)h2, st, d_out);
    return hipGetLastError();
}

}  // extern "C"
