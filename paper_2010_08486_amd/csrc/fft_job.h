// One job of the transform-domain blur (device code), shared by the
// transform kernel of dct.hip and the blur kernels of kernels.hip, which run
// such jobs in the same launch as their direct tiles.  Not part of the
// public C ABI.
//
// A job blurs two lines u1, u2 of N = 2^LOGN values (consecutive rows or
// columns of its input) by the kernels of its planes, as products in the type-II cosine
// transform domain (exact for the half-sample symmetric border; the module
// comment of dct.hip gives the transforms):
//   1. load both lines as z = v1 + i v2, v the even/odd reordering of u, at
//      bit-reversed positions in LDS;
//   2. forward FFT;
//   3. for each pair of frequencies (k, N-k), the cosine coefficients of both
//      lines, kept in registers;
//   4. per plane: scale by the plane's transfer function (H/N), form the
//      inverse sequence, inverse FFT, store both lines as rows of the plane.
// Every global load of a phase is issued before the first is waited for
// (loop bounds are compile-time constants; loads past the end read a valid
// element again, so no load sits in a branch).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dct.h"
#include "dog_internal.h"

// Pointers into the global address space, and into memory no kernel
// writes (loads through the latter may go through the scalar cache when
// every lane reads the same address).  The qualifiers only exist for the
// device compilation pass; the host pass sees plain pointers.
#if defined(__HIP_DEVICE_COMPILE__)
#define DOG_GLOBAL_AS __attribute__((address_space(1)))
#define DOG_CONST_AS __attribute__((address_space(4)))   // read-only for the kernel
#else
#define DOG_GLOBAL_AS
#define DOG_CONST_AS
#endif

namespace dog {
namespace fftd {

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

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
#pragma clang fp contract(on)
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int LOGN>
__device__ __forceinline__ uint32_t bitrev(uint32_t v)
{
    return __builtin_bitreverse32(v) >> (32 - LOGN);
}

// Position of element n of a line after the even/odd reordering.
__device__ __forceinline__ uint32_t reorder(uint32_t n, uint32_t N)
{
    return (n & 1u) ? N - 1u - (n >> 1) : (n >> 1);
}

// LDS position of element i of the sequence: one float2 of padding after
// every 16, so the power-of-two strides of the FFT stages and of the
// bit-reversed placement spread over the banks.
__device__ __forceinline__ uint32_t pd(uint32_t i) { return i + (i >> 4); }

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

// In-place FFT of one sequence of N complex values in LDS (input at
// bit-reversed positions, output in natural order) by NT threads: the
// radix-2 decimation-in-time stages, taken two at a time from registers
// (each thread loads four elements i, i+h, i+2h, i+3h of a block of 4h,
// applies stage s to the pairs (i, i+h), (i+2h, i+3h) and stage s+1 to
// (i, i+2h), (i+h, i+3h), and stores them), then a last single stage when
// log2 N is odd.  tw[t] = exp(-2 pi i t / N); INV conjugates the twiddles
// (no 1/N).  Every shift and mask is a constant.
template <bool INV, int LOGN, int NT>
__device__ __forceinline__ void fft_seq(float2* buf, const float2* tw)
{
    constexpr uint32_t groups = 1u << (LOGN - 2);   // blocks of 4 elements
#pragma unroll
    for (int s = 0; s + 1 < LOGN; s += 2) {
        const uint32_t h = 1u << s;
#pragma unroll
        for (uint32_t g0 = 0; g0 < groups; g0 += NT) {
            const uint32_t j = g0 + threadIdx.x;
            if (groups % NT == 0 || j < groups) {
                const uint32_t q = j & (h - 1u);
                const uint32_t i0 = ((j >> s) << (s + 2)) + q;
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
        for (uint32_t g0 = 0; g0 < half; g0 += NT) {
            const uint32_t q = g0 + threadIdx.x;
            if (half % NT == 0 || q < half) {
                float2 a = buf[pd(q)], b = buf[pd(q + half)];
                bfly(a, b, twid<INV>(tw, q));
                buf[pd(q)] = a;
                buf[pd(q + half)] = b;
            }
        }
        __syncthreads();
    }
}

}  // namespace fftd

// Sizes of a job of lines of 2^LOGN values run by NT threads.
template <int LOGN, int NT>
struct FftGeom {
    static constexpr uint32_t N = 1u << LOGN;
    static constexpr uint32_t HALF = N / 2;
    static constexpr int LOADS = (int)((N + NT - 1) / NT);             // rows per thread
    static constexpr uint32_t ITEMS = HALF + 1;                        // (k, N-k) pairs
    static constexpr int IPT = (int)((ITEMS + NT - 1) / NT);           // pairs per thread
    static constexpr int TW = (int)((HALF + NT - 1) / NT);
    static constexpr uint32_t SEQ = N + N / 16;                        // padded sequence
    // LDS: the padded sequence, N/2 twiddles, N post-twiddles
    static constexpr size_t LDS_BYTES = (size_t)(SEQ + HALF + N) * sizeof(float2);
};

// The job at jp, run by the NT threads of the workgroup with `lds` (at least
// FftGeom::LDS_BYTES, 8-byte aligned).  VEC: the input rows hold a column
// job's two lines at 8-byte aligned addresses.  Returns at once for a job with no
// planes (padding); every barrier is reached by all NT threads otherwise.
template <int LOGN, int NT, bool VEC>
__device__ __forceinline__ void fft_job(const LaunchArgs& a, const FftJob* __restrict__ jp,
                                        float2* lds)
{
    using namespace fftd;
    using G = FftGeom<LOGN, NT>;
    constexpr uint32_t N = G::N, half = G::HALF;
    static_assert(kFftLines == 2, "one complex sequence per job");
    const int n_planes = jp->n_planes;
    if (n_planes <= 0)
        return;
    // the job's fields, read once (stores through the output pointers could
    // otherwise make the compiler read them again after every store)
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
    const bool in_rows = jp->in_rows != 0;
    const size_t out_pitch = (size_t)jp->out_pitch;
    const auto tw_g = gptr(jp->tw);
    const auto post_g = gptr(jp->post);
    float2* buf = lds;              // the sequence, at pd(i)
    float2* tw = lds + G::SEQ;      // N/2 twiddles
    float2* post = tw + half;       // N post-twiddles exp(-i pi k / (2N))
    const uint32_t tid = threadIdx.x;

    // ---- every load of the first phase at once
    float2 v[G::LOADS];
    const auto in_g = gptr(in);
#pragma unroll
    for (int q = 0; q < G::LOADS; ++q) {
        const uint32_t n = min(tid + (uint32_t)q * NT, N - 1u);
        if (in_rows) {
            const size_t o = (size_t)line0 * pitch + n;
            v[q] = make_float2(in_g[o], in_g[o + pitch]);
        } else {
            const size_t o = (size_t)n * pitch + line0;
            if (VEC)
                v[q] = *reinterpret_cast<const DOG_GLOBAL_AS float2*>(in_g + o);
            else
                v[q] = make_float2(in_g[o], in_g[o + 1]);
        }
    }
    float2 twr[G::TW], pr[G::LOADS];
#pragma unroll
    for (int q = 0; q < G::TW; ++q)
        twr[q] = tw_g[min(tid + (uint32_t)q * NT, half - 1u)];
#pragma unroll
    for (int q = 0; q < G::LOADS; ++q)
        pr[q] = post_g[min(tid + (uint32_t)q * NT, N - 1u)];
    float hk[G::IPT], hm[G::IPT];
    auto load_h = [&](const float* h) {
        const auto hg = gptr(h);
#pragma unroll
        for (int q = 0; q < G::IPT; ++q) {
            const uint32_t k = min(tid + (uint32_t)q * NT, half);
            hk[q] = hg[k];
            hm[q] = hg[(N - k) & (N - 1u)];
        }
    };
    const FftPlaneSet* __restrict__ ps = jp->planes;
    load_h(ps->h[0]);
#pragma unroll
    for (int q = 0; q < G::TW; ++q)
        if (tid + (uint32_t)q * NT < half)
            tw[tid + q * NT] = twr[q];
#pragma unroll
    for (int q = 0; q < G::LOADS; ++q) {
        const uint32_t n = tid + (uint32_t)q * NT;
        if (n < N) {
            post[n] = pr[q];
            buf[pd(bitrev<LOGN>(reorder(n, N)))] = v[q];
        }
    }
    __syncthreads();   // the lines, twiddles and post-twiddles are in LDS
    fft_seq<false, LOGN, NT>(buf, tw);

    // ---- cosine coefficients of both lines at k and N-k:
    // V1 = (Z[k] + conj Z[N-k]) / 2, V2 = (Z[k] - conj Z[N-k]) / (2i),
    // C[k] = Re(exp(-i pi k / (2N)) V[k]), and V[N-k] = conj V[k]
    float c1k[G::IPT], c2k[G::IPT], c1m[G::IPT], c2m[G::IPT];
#pragma unroll
    for (int q = 0; q < G::IPT; ++q) {
        const uint32_t k = min(tid + (uint32_t)q * NT, half);
        const uint32_t m = (N - k) & (N - 1u);
        const float2 z = buf[pd(k)], zm = buf[pd(m)];
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
        const auto out = gptr_w(ps->out[pl]);
        // ---- inverse sequence: per line V[k] = exp(i pi k / (2N)) (H_k C_k -
        // i H_{N-k} C_{N-k}), both lines as Z = V1 + i V2
#pragma unroll
        for (int q = 0; q < G::IPT; ++q) {
            const uint32_t k = tid + (uint32_t)q * NT;
            if (k <= half) {
                const uint32_t m = (N - k) & (N - 1u);
                const float a1 = c1k[q] * hk[q], b1 = c1m[q] * hm[q];
                const float a2 = c2k[q] * hk[q], b2 = c2m[q] * hm[q];
                const float2 ek = post[k];
                const float ck = ek.x, sk = -ek.y;
                const float2 V1 = make_float2(ck * a1 + sk * b1, sk * a1 - ck * b1);
                const float2 V2 = make_float2(ck * a2 + sk * b2, sk * a2 - ck * b2);
                buf[pd(bitrev<LOGN>(k))] = make_float2(V1.x - V2.y, V1.y + V2.x);
                if (k != 0 && k != half) {
                    const float2 em = post[m];
                    const float cm = em.x, sm = -em.y;
                    const float2 W1 = make_float2(cm * b1 + sm * a1, sm * b1 - cm * a1);
                    const float2 W2 = make_float2(cm * b2 + sm * a2, sm * b2 - cm * a2);
                    buf[pd(bitrev<LOGN>(m))] = make_float2(W1.x - W2.y, W1.y + W2.x);
                }
            }
        }
        if (pl + 1 < n_planes)   // the next plane's transfer function, in flight
            load_h(ps->h[pl + 1]);
        __syncthreads();
        fft_seq<true, LOGN, NT>(buf, tw);

        // ---- store: u[2n] = v[n], u[2n+1] = v[N-1-n] per line; the two
        // lines are rows line0 and line0 + 1 of the plane
#pragma unroll
        for (int q = 0; q < G::LOADS; ++q) {
            const uint32_t n = tid + (uint32_t)q * NT;
            if (n < half) {
                const float2 x = buf[pd(n)], y = buf[pd(N - 1u - n)];
                const size_t o = (size_t)line0 * out_pitch + 2 * n;
                *reinterpret_cast<DOG_GLOBAL_AS float2*>(out + o) = make_float2(x.x, y.x);
                *reinterpret_cast<DOG_GLOBAL_AS float2*>(out + o + out_pitch) =
                    make_float2(x.y, y.y);
            }
        }
        __syncthreads();   // the buffer is refilled by the next plane
    }
}

}  // namespace dog
