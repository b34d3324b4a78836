// Transform-domain blur of the widest ladder planes (Sec. 4.1: the blur as a
// convolution that can also be taken through a fast Fourier transform,
// whose cost does not grow with sigma).
//
// The half-sample symmetric reflection the direct blur uses at the borders
// is the even extension of period 2N that the type-II discrete cosine
// transform diagonalises: for a line u of length N,
//     C[k] = sum_n u[n] cos(pi k (2n + 1) / (2N)),   k = 0..N-1,
// and the blur of u by a symmetric kernel w (any radius; wraps of the period
// are included) has the transform H[k] C[k] with
//     H[k] = sum_{j=-r..r} w_j cos(pi k j / N).
// So each of the two separable blur passes of such a plane is, line by line,
// a forward cosine transform, a product with H, and an inverse transform,
// exact up to rounding.
//
// Each 1-D transform of length N (a power of two) goes through one complex
// FFT of length N for two real lines at once (z = u1 + i u2), after the
// even/odd reordering that turns the cosine transform into a Fourier one:
//     v[n] = u[2n], v[N-1-n] = u[2n+1];  C[k] = Re(exp(-i pi k/(2N)) V[k]),
// and, inversely, V[k] = exp(i pi k/(2N)) (C[k] - i C[N-k]) (C[N] = 0),
// v = sum_k V[k] exp(2 pi i k n / N), u[2n] = v[n], u[2n+1] = v[N-1-n]
// (the 1/N of the inverse is folded into the transfer functions).  The FFT
// runs in LDS: radix-2 decimation in time, stages taken two at a time, in
// place, the input placed at bit-reversed positions as it is loaded.
// Twiddles and transfer functions are FP64 values rounded once to fp32, from
// host tables.
//
// A workgroup blurs four lines that are consecutive columns of its input
// (two complex sequences) and produces, from one forward transform, the
// lines of every plane the job lists.  The two launches of a frame:
//   pass 1: the columns of the frame X[y][x] (lines along y), one forward
//           transform, then every transform-domain plane p, each output line
//           a row of T_p (the transposed layout of the direct pass 1);
//   pass 2: per plane, the columns of T_p (lines along x), output lines
//           columns of L_p, the layout of the direct pass 2.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "dct.h"

namespace dog {

namespace {

constexpr int kNT = 512;   // threads per job: eight waves, two per SIMD

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ uint32_t bitrev(uint32_t v, int logn)
{
    return __builtin_bitreverse32(v) >> (32 - logn);
}

// Position of element n of a line after the even/odd reordering.
__device__ __forceinline__ uint32_t reorder(uint32_t n, uint32_t N)
{
    return (n & 1u) ? N - 1u - (n >> 1) : (n >> 1);
}

// LDS position of element i of the sequences: one float2 of padding after
// every 16, so the power-of-two strides of the FFT stages and of the
// bit-reversed placement spread over the banks.
__device__ __forceinline__ uint32_t pd(uint32_t i) { return i + (i >> 4); }

// In-place FFT of two sequences of N complex values in LDS (input at
// bit-reversed positions, output in natural order): the radix-2
// decimation-in-time stages, taken two at a time from registers (each
// thread loads four elements i, i+h, i+2h, i+3h of a block of 4h, applies
// stage s to the pairs (i, i+h), (i+2h, i+3h) and stage s+1 to (i, i+2h),
// (i+h, i+3h), and stores them), then a last single stage when log2 N is
// odd.  tw[t] = exp(-2 pi i t / N); INV conjugates the twiddles (no 1/N).
template <bool INV>
__device__ __forceinline__ float2 twid(const float2* tw, uint32_t t)
{
    float2 w = tw[t];
    if (INV)
        w.y = -w.y;
    return w;
}

__device__ __forceinline__ void bfly(float2& a, float2& b, float2 w)
{
    const float2 t = cmul(w, b);
    b = make_float2(a.x - t.x, a.y - t.y);
    a = make_float2(a.x + t.x, a.y + t.y);
}

template <bool INV, int LOGN>
__device__ __forceinline__ void fft_pair(float2* buf, const float2* tw)
{
    constexpr uint32_t groups = 1u << (LOGN - 1);   // blocks of 4 elements, both sequences
    // stage pairs (s, s + 1); every shift and mask below is a constant
#pragma unroll
    for (int s = 0; s + 1 < LOGN; s += 2) {
        const uint32_t h = 1u << s;
#pragma unroll
        for (uint32_t g0 = 0; g0 < groups; g0 += kNT) {
            const uint32_t g = g0 + threadIdx.x;
            if (groups % kNT == 0 || g < groups) {
                const uint32_t p = g >> (LOGN - 2);
                const uint32_t j = g & ((1u << (LOGN - 2)) - 1u);
                const uint32_t q = j & (h - 1u);
                const uint32_t i0 = (p << LOGN) + ((j >> s) << (s + 2)) + q;
                float2 a0 = buf[pd(i0)], a1 = buf[pd(i0 + h)], a2 = buf[pd(i0 + 2 * h)],
                       a3 = buf[pd(i0 + 3 * h)];
                const float2 w1 = twid<INV>(tw, q << (LOGN - s - 1));
                bfly(a0, a1, w1);
                bfly(a2, a3, w1);
                bfly(a0, a2, twid<INV>(tw, q << (LOGN - s - 2)));
                bfly(a1, a3, twid<INV>(tw, (q + h) << (LOGN - s - 2)));
                buf[pd(i0)] = a0;
                buf[pd(i0 + h)] = a1;
                buf[pd(i0 + 2 * h)] = a2;
                buf[pd(i0 + 3 * h)] = a3;
            }
        }
        __syncthreads();
    }
    if (LOGN % 2) {   // the last stage on its own: pairs (q, q + N/2)
        constexpr uint32_t half = 1u << (LOGN - 1);
#pragma unroll
        for (uint32_t g0 = 0; g0 < 2 * groups; g0 += kNT) {
            const uint32_t g = g0 + threadIdx.x;
            if ((2 * groups) % kNT == 0 || g < 2 * groups) {
                const uint32_t p = g >> (LOGN - 1);
                const uint32_t q = g & (half - 1u);
                const uint32_t i0 = (p << LOGN) + q;
                float2 a = buf[pd(i0)], b = buf[pd(i0 + half)];
                bfly(a, b, twid<INV>(tw, q));
                buf[pd(i0)] = a;
                buf[pd(i0 + half)] = b;
            }
        }
        __syncthreads();
    }
}

}  // namespace

// Pointers into the global address space.  The qualifier only exists for
// the device compilation pass; the host pass of this file sees plain
// pointers.
#if defined(__HIP_DEVICE_COMPILE__)
#define DOG_GLOBAL_AS __attribute__((address_space(1)))
#else
#define DOG_GLOBAL_AS
#endif

// Global-memory views of pointers the job table holds (the compiler cannot
// tell their address space, and generic loads would also wait on LDS).
template <class T>
__device__ __forceinline__ const DOG_GLOBAL_AS T* gptr(const T* p)
{
    return (const DOG_GLOBAL_AS T*)p;
}
template <class T>
__device__ __forceinline__ DOG_GLOBAL_AS T* gptr_w(T* p)
{
    return (DOG_GLOBAL_AS T*)p;
}

// Blur of one job's lines (module comment), lines of N = 2^LOGN values: load
// the kFftLines lines as two complex sequences in even/odd order at
// bit-reversed positions, forward FFT, cosine coefficients of both lines for
// each pair of frequencies (k, N-k) kept in registers, then per plane: scale
// by the plane's transfer function, form the inverse sequence, inverse FFT,
// store the lines.  Every global load of a phase is issued before the first
// is waited for (loop bounds are compile-time constants and loads past the
// end read a valid element again, so no load sits in a branch): the lines,
// twiddles and the first plane's transfer function together, and each later
// plane's transfer function during the previous plane's inverse.
// Dynamic LDS: 2 padded sequences of N float2, N/2 twiddles, N post-twiddles.
static_assert(kFftLines == 4, "two complex sequences per job");

template <int LOGN>
struct FftGeom {
    static constexpr uint32_t N = 1u << LOGN;
    static constexpr uint32_t HALF = N / 2;
    static constexpr int LOADS = (int)((N + kNT - 1) / kNT);             // rows per thread
    static constexpr uint32_t ITEMS = 2 * (HALF + 1);                    // (k, N-k) pairs
    static constexpr int IPT = (int)((ITEMS + kNT - 1) / kNT);           // pairs per thread
    static constexpr int TW = (int)((HALF + kNT - 1) / kNT);
    static constexpr uint32_t SEQ = N * 2 + (N * 2) / 16;                // padded sequences
};

template <int LOGN>
__device__ __forceinline__ void pair_index(uint32_t i, uint32_t& p, uint32_t& k, uint32_t& m)
{
    using G = FftGeom<LOGN>;
    p = i >= G::HALF + 1 ? 1u : 0u;
    k = i - p * (G::HALF + 1);
    m = (G::N - k) & (G::N - 1u);
}

// Transfer function values H[k], H[N-k] of this thread's pairs.
template <int LOGN>
__device__ __forceinline__ void load_h(float (&hk)[FftGeom<LOGN>::IPT],
                                       float (&hm)[FftGeom<LOGN>::IPT], const float* h,
                                       uint32_t tid)
{
    using G = FftGeom<LOGN>;
    const auto hg = gptr(h);
#pragma unroll
    for (int q = 0; q < G::IPT; ++q) {
        const uint32_t i = min(tid + (uint32_t)q * kNT, G::ITEMS - 1u);
        uint32_t p, k, m;
        pair_index<LOGN>(i, p, k, m);
        hk[q] = hg[k];
        hm[q] = hg[m];
    }
}

template <int LOGN, bool VEC>
__global__ void __launch_bounds__(kNT) k_fft_blur(LaunchArgs a, const FftJob* __restrict__ jobs)
{
    using G = FftGeom<LOGN>;
    constexpr uint32_t N = G::N, half = G::HALF;
    extern __shared__ __align__(16) float2 lds[];
    // the job's fields, read once (stores through the output pointers could
    // otherwise make the compiler read them again after every store)
    const FftJob* __restrict__ jp = jobs + blockIdx.x;
    const float* in = jp->in;
    long long pitch = jp->in_pitch;
    if (!in) {
        // the frame's own pixels (their pointer changes between launches of
        // the same tables; the descriptor carries it)
        const FrameDesc& f = a.frames ? a.frames[jp->frame] : a.f0;
        in = f.src;
        pitch = f.src_stride;
    }
    const uint32_t line0 = (uint32_t)jp->line0;
    const int n_planes = jp->n_planes;
    const bool out_rows = jp->out_rows != 0;
    const size_t out_pitch = (size_t)jp->out_pitch;
    const auto tw_g = gptr(jp->tw);
    const auto post_g = gptr(jp->post);
    float2* buf = lds;              // sequence p at buf + pd(p * N + i)
    float2* tw = lds + G::SEQ;      // N/2 twiddles
    float2* post = tw + half;       // N post-twiddles exp(-i pi k / (2N))
    const uint32_t tid = threadIdx.x;

    // ---- every load of the first phase at once: row n holds the four lines'
    // values at position n (lines 0, 1: sequence 0; lines 2, 3: sequence 1)
    float4 v[G::LOADS];
    const auto in_g = gptr(in);
#pragma unroll
    for (int q = 0; q < G::LOADS; ++q) {
        const uint32_t n = min(tid + (uint32_t)q * kNT, N - 1u);
        const size_t o = (size_t)n * pitch + line0;
        if (VEC) {
            v[q] = *reinterpret_cast<const DOG_GLOBAL_AS float4*>(in_g + o);
        } else {
            v[q] = make_float4(in_g[o], in_g[o + 1], in_g[o + 2], in_g[o + 3]);
        }
    }
    float2 twr[G::TW], pr[G::LOADS];
#pragma unroll
    for (int q = 0; q < G::TW; ++q)
        twr[q] = tw_g[min(tid + (uint32_t)q * kNT, half - 1u)];
#pragma unroll
    for (int q = 0; q < G::LOADS; ++q)
        pr[q] = post_g[min(tid + (uint32_t)q * kNT, N - 1u)];
    float hk[G::IPT], hm[G::IPT];
    load_h<LOGN>(hk, hm, jp->h[0], tid);
#pragma unroll
    for (int q = 0; q < G::TW; ++q)
        if (tid + (uint32_t)q * kNT < half)
            tw[tid + q * kNT] = twr[q];
#pragma unroll
    for (int q = 0; q < G::LOADS; ++q) {
        const uint32_t n = tid + (uint32_t)q * kNT;
        if (n < N) {
            post[n] = pr[q];
            const uint32_t pos = bitrev(reorder(n, N), LOGN);
            buf[pd(pos)] = make_float2(v[q].x, v[q].y);
            buf[pd(N + pos)] = make_float2(v[q].z, v[q].w);
        }
    }
    __syncthreads();   // the lines, twiddles and post-twiddles are in LDS
    fft_pair<false, LOGN>(buf, tw);

    // ---- cosine coefficients of both lines of each sequence at k and N-k:
    // V1 = (Z[k] + conj Z[N-k]) / 2, V2 = (Z[k] - conj Z[N-k]) / (2i),
    // C[k] = Re(exp(-i pi k / (2N)) V[k]), and V[N-k] = conj V[k]
    float c1k[G::IPT], c2k[G::IPT], c1m[G::IPT], c2m[G::IPT];
#pragma unroll
    for (int q = 0; q < G::IPT; ++q) {
        const uint32_t i = min(tid + (uint32_t)q * kNT, G::ITEMS - 1u);
        uint32_t p, k, m;
        pair_index<LOGN>(i, p, k, m);
        const float2 z = buf[pd(p * N + k)], zm = buf[pd(p * N + m)];
        const float2 V1 = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
        const float2 V2 = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));
        const float2 ek = post[k], em = post[m];   // (cos, -sin) of pi k / (2N)
        c1k[q] = ek.x * V1.x - ek.y * V1.y;
        c2k[q] = ek.x * V2.x - ek.y * V2.y;
        c1m[q] = k ? em.x * V1.x + em.y * V1.y : 0.0f;   // Re(e_m conj V1); C_N = 0
        c2m[q] = k ? em.x * V2.x + em.y * V2.y : 0.0f;
    }
    __syncthreads();   // every coefficient read before the buffer is reused

    for (int pl = 0; pl < n_planes; ++pl) {
        const auto out = gptr_w(jp->out[pl]);
        // ---- inverse sequence: per line V[k] = exp(i pi k / (2N)) (H_k C_k -
        // i H_{N-k} C_{N-k}), both lines as Z = V1 + i V2
#pragma unroll
        for (int q = 0; q < G::IPT; ++q) {
            const uint32_t i = tid + (uint32_t)q * kNT;
            if (i < G::ITEMS) {
                uint32_t p, k, m;
                pair_index<LOGN>(i, p, k, m);
                const float a1 = c1k[q] * hk[q], b1 = c1m[q] * hm[q];
                const float a2 = c2k[q] * hk[q], b2 = c2m[q] * hm[q];
                const float2 ek = post[k];
                const float ck = ek.x, sk = -ek.y;
                const float2 V1 = make_float2(ck * a1 + sk * b1, sk * a1 - ck * b1);
                const float2 V2 = make_float2(ck * a2 + sk * b2, sk * a2 - ck * b2);
                buf[pd(p * N + bitrev(k, LOGN))] = make_float2(V1.x - V2.y, V1.y + V2.x);
                if (k != 0 && k != half) {
                    const float2 em = post[m];
                    const float cm = em.x, sm = -em.y;
                    const float2 W1 = make_float2(cm * b1 + sm * a1, sm * b1 - cm * a1);
                    const float2 W2 = make_float2(cm * b2 + sm * a2, sm * b2 - cm * a2);
                    buf[pd(p * N + bitrev(m, LOGN))] = make_float2(W1.x - W2.y, W1.y + W2.x);
                }
            }
        }
        if (pl + 1 < n_planes)   // the next plane's transfer function, in flight
            load_h<LOGN>(hk, hm, jp->h[pl + 1], tid);
        __syncthreads();
        fft_pair<true, LOGN>(buf, tw);

        // ---- store: u[2n] = v[n], u[2n+1] = v[N-1-n] per line
        if (out_rows) {
            // line l of the job is row line0 + l of the plane
#pragma unroll
            for (int q = 0; q < G::LOADS; ++q) {
                const uint32_t e = tid + (uint32_t)q * kNT;
                if (e < N) {
                    const uint32_t p = e >= half ? 1u : 0u;
                    const uint32_t n = e - p * half;
                    const float2 x = buf[pd(p * N + n)], y = buf[pd(p * N + N - 1u - n)];
                    const size_t o = (size_t)(line0 + 2 * p) * out_pitch + 2 * n;
                    *reinterpret_cast<DOG_GLOBAL_AS float2*>(out + o) =
                        make_float2(x.x, y.x);
                    *reinterpret_cast<DOG_GLOBAL_AS float2*>(out + o + out_pitch) =
                        make_float2(x.y, y.y);
                }
            }
        } else {
            // position n of the four lines is one 16-byte piece of row n
#pragma unroll
            for (int q = 0; q < G::LOADS; ++q) {
                const uint32_t n = tid + (uint32_t)q * kNT;
                if (n < N) {
                    const uint32_t idx = (n & 1u) ? N - 1u - (n >> 1) : (n >> 1);
                    const float2 s0 = buf[pd(idx)], s1 = buf[pd(N + idx)];
                    *reinterpret_cast<DOG_GLOBAL_AS float4*>(
                        out + (size_t)n * out_pitch + line0) = make_float4(s0.x, s0.y, s1.x, s1.y);
                }
            }
        }
        __syncthreads();   // the buffer is refilled by the next plane
    }
}

// The k_fft_blur instance for lines of 2^LOGN values.
template <int LOGN>
const void* fft_fn(int vec)
{
    return vec ? reinterpret_cast<const void*>(&k_fft_blur<LOGN, true>)
               : reinterpret_cast<const void*>(&k_fft_blur<LOGN, false>);
}

}  // namespace dog

extern "C" {

size_t dogk_fft_lds_bytes(int N)
{
    const size_t seq = (size_t)2 * N + (size_t)2 * N / 16;   // padded sequences
    return (seq + (size_t)N / 2 + (size_t)N) * sizeof(float2);
}

hipError_t dogk_fft_blur(const dog::LaunchArgs* args, const dog::FftJob* d_jobs, int n_jobs,
                         int logn, int vec, hipStream_t stream, hipEvent_t* ev)
{
    if (n_jobs <= 0)
        return hipSuccess;
    if (logn < 6 || logn > 11)
        return hipErrorInvalidValue;
    const void* const table[6] = {dog::fft_fn<6>(vec),  dog::fft_fn<7>(vec),
                                  dog::fft_fn<8>(vec),  dog::fft_fn<9>(vec),
                                  dog::fft_fn<10>(vec), dog::fft_fn<11>(vec)};
    const void* fn = table[logn - 6];
    const size_t lds_bytes = dogk_fft_lds_bytes(1 << logn);
    static size_t allowed[6][2] = {};   // dynamic LDS each instance has been allowed
    if (lds_bytes > allowed[logn - 6][vec ? 1 : 0]) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds_bytes);
        if (e != hipSuccess)
            return e;
        allowed[logn - 6][vec ? 1 : 0] = lds_bytes;
    }
    const dog::FftJob* jobs = d_jobs;
    void* params[] = {const_cast<dog::LaunchArgs*>(args), &jobs};
    return ev ? hipExtLaunchKernel(fn, dim3(n_jobs), dim3(dog::kNT), params, lds_bytes, stream,
                                   ev[0], ev[1], 0)
              : hipLaunchKernel(fn, dim3(n_jobs), dim3(dog::kNT), params, lds_bytes, stream);
}

}  // extern "C"
