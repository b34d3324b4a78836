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
// Smoothing: one workgroup per 256 x 8 output tile; each thread blurs its
// input column along y in registers, the results go to LDS, then each
// thread blurs its rows along x into the output (taps in ascending order,
// fp32 FMAs).
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
#include <mutex>

namespace dogpre {

constexpr int kSR = 8;         // output rows per smoothing workgroup (256 columns)
constexpr int kMaxR = 16;      // largest smoothing radius (sigma < 4.125 at truncate 4)
constexpr int kRep = 8;        // replicas of every digit histogram
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
// Each histogram of nb bins is followed by its nb/32 sums of 32 bins, so a
// pick reads 32-bin sums and then one block of 32 bins, not the whole
// histogram (every workgroup picks; whole histograms made them crowd the
// few L2 channels holding them).  Every histogram is kept in kRep replicas
// (a workgroup adds to replica wg % kRep, a pick sums them), so the hot
// bins and sums take kRep times fewer global atomics per address: the
// values of a frame crowd into few digits, and every workgroup adds to them.
constexpr int hwords(int nb) { return nb + nb / 32; }
constexpr size_t kOffH0 = 256;
constexpr size_t kOffH1 = kOffH0 + (size_t)kRep * hwords(kBins) * 4;
constexpr size_t kOffH2 = kOffH1 + 2 * (size_t)kRep * hwords(kBins) * 4;
constexpr size_t kScratch = kOffH2 + 2 * (size_t)kRep * hwords(1024) * 4;

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

// Run by one whole wave: the digit whose bin holds the rank-th smallest key
// (0-based) of an nb-bin histogram (nb = 1024 or 2048) stored as bins then
// 32-bin sums, in `reps` replicas to be added, and the rank within that
// bin; both reach every lane.  The
// sums locate the block of 32 bins, then the bins of that block the digit.
__device__ void wave_pick(const uint32_t* __restrict__ hist, int nb, int reps, uint32_t rank,
                          uint32_t* digit, uint32_t* rem)
{
    const int lane = threadIdx.x & 63;
    const int nc = nb / 32;
    uint32_t cv = 0u;   // summed over the histogram's replicas
    if (lane < nc)
        for (int q = 0; q < reps; ++q)
            cv += hist[q * hwords(nb) + nb + lane];
    uint32_t inc = cv;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)inc, off);
        if (lane >= off)
            inc += v;
    }
    const uint32_t before = inc - cv;
    const unsigned long long who = __ballot(lane < nc && rank >= before && rank < inc);
    const int blk = who ? __builtin_ctzll(who) : 0;
    const uint32_t r2 = rank - (uint32_t)__builtin_amdgcn_readlane((int)before, blk);
    uint32_t fv = 0u;
    if (lane < 32)
        for (int q = 0; q < reps; ++q)
            fv += hist[q * hwords(nb) + blk * 32 + lane];
    uint32_t inc2 = fv;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)inc2, off);
        if (lane >= off)
            inc2 += v;
    }
    const uint32_t before2 = inc2 - fv;
    const unsigned long long who2 = __ballot(lane < 32 && r2 >= before2 && r2 < inc2);
    const int j = who2 ? __builtin_ctzll(who2) : 0;
    *digit = (uint32_t)(blk * 32 + j);
    *rem = r2 - (uint32_t)__builtin_amdgcn_readlane((int)before2, j);
}

// Adds the workgroup's LDS histograms h (nt targets of nb bins) to the
// global ones at g (target t at g + t tstride words): the nonzero bins, then
// the nonzero 32-bin sums.
__device__ void flush_hist(const uint32_t* h, int nt, int nb, uint32_t* g, int tstride)
{
    const int nc = nb / 32;
    for (int i = threadIdx.x; i < nt * nb; i += blockDim.x)
        if (h[i]) {
            const int t = i / nb;
            atomicAdd(&g[t * tstride + (i - t * nb)], h[i]);
        }
    for (int i = threadIdx.x; i < nt * nc; i += blockDim.x) {
        const int t = i / nc, c = i - t * nc;
        uint32_t sum = 0;
        for (int q = 0; q < 32; ++q)
            sum += h[t * nb + c * 32 + q];
        if (sum)
            atomicAdd(&g[t * tstride + nb + c], sum);
    }
}

// Smoothing of a tile of 256 columns x kSR rows at radius R (one column per
// thread; R = 0 with the single weight 1 copies), and the pass-0 digit
// histogram of the smoothed values.  Each thread loads its input column over
// the tile's rows and halo (coalesced along the wave, all loads issued
// before the first use), blurs it along y in registers, and puts the kSR
// results in LDS; threads t < 2R do the same for the right halo columns.
// Then each thread blurs its kSR rows along x from LDS.  R is a template
// argument so that every tap loop unrolls: the LDS reads of a row are issued
// back to back and the weights sit in scalar registers.  The histogram goes
// to one of kRep replicas of hist0 (by workgroup).
template <int R>
__global__ void __launch_bounds__(256) k_smooth(const float* __restrict__ in, int H, int W,
                                                long long stride, const float* __restrict__ w,
                                                float* __restrict__ out,
                                                uint32_t* __restrict__ hist0,
                                                uint32_t* __restrict__ hist1)
{
    constexpr int TW = 256 + 2 * R, TH = kSR + 2 * R, NT = 2 * R + 1;
    __shared__ float tile[kSR * TW];
    __shared__ uint32_t h[kBins];
    const int t = threadIdx.x;
    const int x0 = blockIdx.x * 256, y0 = blockIdx.y * kSR;
    for (int i = t; i < kBins; i += 256)
        h[i] = 0u;
    // the pass-1 histograms must be zero before the next kernel counts
    const int wg = blockIdx.y * gridDim.x + blockIdx.x;
    for (int i = wg * 256 + t; i < 2 * kRep * hwords(kBins); i += gridDim.x * gridDim.y * 256)
        hist1[i] = 0u;
    float wr[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j)
        wr[j] = w[j];
    // input rows y0 - R .. y0 + kSR + R - 1 of columns x0 - R + t and, for
    // t < 2R, x0 + 256 - R + t
    const int xa = reflect(x0 - R + t, W);
    const bool extra = t < 2 * R;
    const int xb = extra ? reflect(x0 - R + 256 + t, W) : 0;
    float va[TH], vb[TH];
#pragma unroll
    for (int yy = 0; yy < TH; ++yy) {
        const float* rowp = in + (long long)reflect(y0 - R + yy, H) * stride;
        va[yy] = rowp[xa];
        vb[yy] = extra ? rowp[xb] : 0.0f;
    }
    // along y, in registers
#pragma unroll
    for (int o = 0; o < kSR; ++o) {
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < NT; ++j)
            acc = __builtin_fmaf(wr[j], va[o + j], acc);
        tile[o * TW + t] = acc;
    }
    if (extra) {
#pragma unroll
        for (int o = 0; o < kSR; ++o) {
            float acc = 0.0f;
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc = __builtin_fmaf(wr[j], vb[o + j], acc);
            tile[o * TW + 256 + t] = acc;
        }
    }
    __syncthreads();
    // along x, from LDS
    const int x = x0 + t;
#pragma unroll
    for (int o = 0; o < kSR; ++o) {
        const float* p = tile + o * TW + t;
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < NT; ++j)
            acc = __builtin_fmaf(wr[j], p[j], acc);
        const bool valid = y0 + o < H && x < W;
        if (valid)
            out[(long long)(y0 + o) * W + x] = acc;
        wave_hist_add(h, key_of(acc) >> 21, valid);
    }
    __syncthreads();
    flush_hist(h, 1, kBins, hist0 + (size_t)(wg % kRep) * hwords(kBins), 0);
}

using SmoothFn = void (*)(const float*, int, int, long long, const float*, float*, uint32_t*,
                          uint32_t*);

template <int... Rs>
struct SmoothTable {
    static constexpr SmoothFn fn[sizeof...(Rs)] = {&k_smooth<Rs>...};
};

// Keys of the kBatch values of this thread in the batch starting at base.
__device__ __forceinline__ void load_keys(const float* __restrict__ s, long long n, long long base,
                                          uint32_t (&k)[kBatch])
{
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
        const long long i = base + b * blockDim.x + threadIdx.x;
        k[b] = i < n ? key_of(s[i]) : 0u;
    }
}

// Each target's next digit from `hist` (one nb-bin histogram per target in
// `reps` replicas, the target's at stride reps hwords(nb), or one shared
// when `shared`); the results reach every thread through LDS.  Needs at
// least two waves.
__device__ void pick_both(const uint32_t* __restrict__ hist, int nb, int reps, bool shared,
                          const uint32_t rank[2], uint32_t* s_res, uint32_t digit[2],
                          uint32_t rem[2])
{
    const int wave = threadIdx.x >> 6;
    if (wave < 2) {   // waves 0 and 1 pick the two targets side by side
        const int tg = wave;
        uint32_t dg, rm;
        wave_pick(hist + (shared ? 0 : tg * reps * hwords(nb)), nb, reps, rank[tg], &dg, &rm);
        if ((threadIdx.x & 63) == 0) {
            s_res[2 * tg] = dg;
            s_res[2 * tg + 1] = rm;
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
    __shared__ uint32_t h[2 * kBins];
    __shared__ uint32_t s_res[4];
    const uint32_t rk0[2] = {rank_lo, rank_hi};
    uint32_t d0[2], rk[2];
    for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x)
        h[i] = 0u;
    // the first keys are loaded before the pick, so their latency overlaps it
    const long long step = (long long)gridDim.x * blockDim.x * kBatch;
    long long base = (long long)blockIdx.x * blockDim.x * kBatch;
    uint32_t k[kBatch];
    load_keys(s, n, base, k);
    pick_both(hist0, kBins, kRep, true, rk0, s_res, d0, rk);   // ends with a barrier
    if (blockIdx.x == 0 && threadIdx.x < 2) {
        st->prefix[0][threadIdx.x] = d0[threadIdx.x];
        st->rank[0][threadIdx.x] = rk[threadIdx.x];
    }
    // the pass-2 histograms must be zero before the next kernel counts
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 2 * kRep * hwords(1024);
         i += gridDim.x * blockDim.x)
        hist2[i] = 0u;
    for (; base < n; base += step) {
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const bool valid = base + b * blockDim.x + threadIdx.x < n;
            const uint32_t d = (k[b] >> 10) & 0x7ffu;
            wave_hist_add(h, d, valid && (k[b] >> 21) == d0[0]);
            wave_hist_add(h + kBins, d, valid && (k[b] >> 21) == d0[1]);
        }
        if (base + step < n)
            load_keys(s, n, base + step, k);
    }
    __syncthreads();
    flush_hist(h, 2, kBins, hist1 + (size_t)(blockIdx.x % kRep) * hwords(kBins),
               kRep * hwords(kBins));
}

// Pass 2: the second digits from hist1, then the histograms of the low 10
// bits of the keys that share each target's top 22 bits.
__global__ void __launch_bounds__(256) k_select_pass2(const float* __restrict__ s, long long n,
                                                      const uint32_t* __restrict__ hist1,
                                                      uint32_t* __restrict__ hist2,
                                                      SelectState* st)
{
    __shared__ uint32_t h[2 * 1024];
    __shared__ uint32_t s_res[4];
    const uint32_t d0[2] = {st->prefix[0][0], st->prefix[0][1]};
    const uint32_t rk0[2] = {st->rank[0][0], st->rank[0][1]};
    uint32_t d1[2], rk[2], pre[2];
    for (int i = threadIdx.x; i < 2 * 1024; i += blockDim.x)
        h[i] = 0u;
    const long long step = (long long)gridDim.x * blockDim.x * kBatch;
    long long base = (long long)blockIdx.x * blockDim.x * kBatch;
    uint32_t k[kBatch];
    load_keys(s, n, base, k);
    pick_both(hist1, kBins, kRep, false, rk0, s_res, d1, rk);   // ends with a barrier
    for (int tg = 0; tg < 2; ++tg)
        pre[tg] = (d0[tg] << 11) | d1[tg];
    if (blockIdx.x == 0 && threadIdx.x < 2) {
        st->prefix[1][threadIdx.x] = pre[threadIdx.x];
        st->rank[1][threadIdx.x] = rk[threadIdx.x];
    }
    for (; base < n; base += step) {
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const bool valid = base + b * blockDim.x + threadIdx.x < n;
            const uint32_t d = k[b] & 0x3ffu;
            wave_hist_add(h, d, valid && (k[b] >> 10) == pre[0]);
            wave_hist_add(h + 1024, d, valid && (k[b] >> 10) == pre[1]);
        }
        if (base + step < n)
            load_keys(s, n, base + step, k);
    }
    __syncthreads();
    flush_hist(h, 2, 1024, hist2 + (size_t)(blockIdx.x % kRep) * hwords(1024),
               kRep * hwords(1024));
}

// The last digits from hist2 give the limits (workgroup 0 stores them for
// the host), then the stretch.  Each thread takes chunks of 4 consecutive
// values (one 16-byte load and store when both buffers are 16-byte
// aligned); its first chunk is loaded before the pick, so that load's
// latency overlaps it.
__global__ void __launch_bounds__(256) k_stretch(const float* __restrict__ s, long long n,
                                                 uint32_t* __restrict__ hist0,
                                                 const uint32_t* __restrict__ hist2,
                                                 SelectState* st, float* __restrict__ out)
{
    __shared__ uint32_t s_res[4];
    const uint32_t pre[2] = {st->prefix[1][0], st->prefix[1][1]};
    const uint32_t rk1[2] = {st->rank[1][0], st->rank[1][1]};
    uint32_t d2[2], rk[2];
    const bool vec = ((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
    const long long nch = (n + 3) / 4;
    const long long step = (long long)gridDim.x * blockDim.x;
    long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    auto load = [&](long long ch) {
        float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const long long i = 4 * ch;
        if (ch < nch) {
            if (vec && i + 4 <= n) {
                v = *reinterpret_cast<const float4*>(s + i);
            } else {
                v.x = s[i];
                if (i + 1 < n)
                    v.y = s[i + 1];
                if (i + 2 < n)
                    v.z = s[i + 2];
                if (i + 3 < n)
                    v.w = s[i + 3];
            }
        }
        return v;
    };
    float4 v = load(c);
    pick_both(hist2, 1024, kRep, false, rk1, s_res, d2, rk);
    const float lo = value_of((pre[0] << 10) | d2[0]);
    const float hi = value_of((pre[1] << 10) | d2[1]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->limit[0] = lo;
        st->limit[1] = hi;
    }
    // leave the pass-0 histogram zero for the next call's smoothing kernel
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kRep * hwords(kBins);
         i += gridDim.x * blockDim.x)
        hist0[i] = 0u;
    auto stretch = [&](float x) {
        return hi > lo ? fminf(fmaxf((x - lo) / (hi - lo), 0.0f), 1.0f) : 0.0f;
    };
    for (; c < nch; c += step) {
        const float4 x = v;
        if (c + step < nch)
            v = load(c + step);
        const float4 y = make_float4(stretch(x.x), stretch(x.y), stretch(x.z), stretch(x.w));
        const long long i = 4 * c;
        if (vec && i + 4 <= n) {
            *reinterpret_cast<float4*>(out + i) = y;
        } else {
            out[i] = y.x;
            if (i + 1 < n)
                out[i + 1] = y.y;
            if (i + 2 < n)
                out[i + 2] = y.z;
            if (i + 3 < n)
                out[i + 3] = y.w;
        }
    }
}

// Set-up of a call that allocates nothing: clear the select state and the
// histograms (the four kernels expect zero histograms; a fill kernel rather
// than a memset, so the call can be captured into a graph), and put the
// smoothing weights, passed by value, after them.
struct SmoothWeights {
    float w[2 * kMaxR + 1];
};

__global__ void __launch_bounds__(256) k_noalloc_setup(uint32_t* __restrict__ words, int n_words,
                                                       SmoothWeights sw, float* __restrict__ wdst,
                                                       int nw)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += gridDim.x * blockDim.x)
        words[i] = 0u;
    if (blockIdx.x == 0 && (int)threadIdx.x < nw)
        wdst[threadIdx.x] = sw.w[threadIdx.x];
}

__global__ void k_copy_limits(const float* __restrict__ src, float* __restrict__ dst)
{
    if (threadIdx.x < 2)
        dst[threadIdx.x] = src[threadIdx.x];
}

// Bytes of the static scratch: select state and histograms, then the weights.
constexpr size_t kNoAllocWeights = kScratch;
constexpr size_t kNoAllocBytes = kScratch + 256;
static_assert((2 * kMaxR + 1) * sizeof(float) <= 256, "weights fit the scratch tail");

}  // namespace dogpre

// Scratch of the preprocessing variant that allocates nothing: one copy per
// GPU, held until the process ends.  Host code never uses this name as an
// address (on the host it is only a stand-in for the symbol); it uses the
// device address that hipGetSymbolAddress returns for the current GPU.
static __device__ __align__(256) unsigned char scratch[dogpre::kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per GPU
}  // namespace

extern "C" {

hipError_t dogk_preprocess(const float* d_in, int H, int W, long long stride, const float* d_w,
                           int r, float* d_s, float* d_out, void* d_scratch, uint32_t rank_lo,
                           uint32_t rank_hi, hipStream_t stream);

size_t dogk_preprocess_noalloc_bytes() { return dogpre::kNoAllocBytes; }

// Device address of the static scratch on the current GPU, looked up once
// per device (with that device current) and kept.
hipError_t dogk_noalloc_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// dogk_preprocess with its scratch and weights in the static array of the
// current GPU: set-up kernel, the four preprocessing kernels, and (d_limits
// non-NULL) a copy of the two limits to d_limits on the device.  w_host: the
// 2r+1 fp32 weights.  Calls overlapping on one GPU share the array and race.
hipError_t dogk_preprocess_noalloc(const float* d_in, int H, int W, long long stride,
                                   const float* w_host, int r, float* d_s, float* d_out,
                                   float* d_limits, uint32_t rank_lo, uint32_t rank_hi,
                                   hipStream_t stream)
{
    using namespace dogpre;
    if (r < 0 || r > kMaxR)
        return hipErrorInvalidValue;
    void* p = nullptr;
    hipError_t e = dogk_noalloc_scratch(&p);
    if (e != hipSuccess)
        return e;
    char* base = static_cast<char*>(p);
    SmoothWeights sw{};
    for (int j = 0; j <= 2 * r; ++j)
        sw.w[j] = w_host[j];
    float* d_w = reinterpret_cast<float*>(base + kNoAllocWeights);
    hipLaunchKernelGGL(k_noalloc_setup, dim3(64), dim3(256), 0, stream,
                       reinterpret_cast<uint32_t*>(base), (int)(kScratch / 4), sw, d_w, 2 * r + 1);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if ((e = dogk_preprocess(d_in, H, W, stride, d_w, r, d_s, d_out, base, rank_lo, rank_hi,
                             stream)) != hipSuccess)
        return e;
    if (d_limits) {
        hipLaunchKernelGGL(k_copy_limits, dim3(1), dim3(64), 0, stream,
                           reinterpret_cast<const float*>(base + 16), d_limits);
        e = hipGetLastError();
    }
    return e;
}

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
    if (r < 0 || r > kMaxR)
        return hipErrorInvalidValue;
    using Table = SmoothTable<0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16>;
    static_assert(sizeof(Table::fn) / sizeof(Table::fn[0]) == kMaxR + 1, "one kernel per radius");
    const dim3 grid((unsigned)((W + 255) / 256), (unsigned)((H + kSR - 1) / kSR));
    hipLaunchKernelGGL(Table::fn[r], grid, dim3(256), 0, stream, d_in, H, W, stride, d_w, d_s, h0,
                       h1);
    const long long g = std::max<long long>(1, std::min<long long>((n + 2047) / 2048, 4096));
    hipLaunchKernelGGL(k_select_pass1, dim3((unsigned)g), dim3(256), 0, stream, (const float*)d_s,
                       n, (const uint32_t*)h0, h1, h2, rank_lo, rank_hi, st);
    hipLaunchKernelGGL(k_select_pass2, dim3((unsigned)g), dim3(256), 0, stream, (const float*)d_s,
                       n, (const uint32_t*)h1, h2, st);
    const long long gs = std::max<long long>(1, std::min<long long>((n + 1023) / 1024, 4096));   // 4 values per thread
    hipLaunchKernelGGL(k_stretch, dim3((unsigned)gs), dim3(256), 0, stream, (const float*)d_s, n, h0,
                       (const uint32_t*)h2, st, d_out);
    return hipGetLastError();
}

}  // extern "C"
