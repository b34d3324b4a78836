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
// So a plane of the ladder is L = IDCT_y IDCT_x ((H_y H_x^T) . DCT_x DCT_y X),
// exact up to rounding.  The forward transform of the frame is shared by
// every plane taken this way; each plane costs one inverse transform.
//
// Each 1-D transform of length N (a power of two) goes through one complex
// FFT of length N for two real lines at once (z = u1 + i u2), after the
// even/odd reordering that turns the cosine transform into a Fourier one:
//     v[n] = u[2n], v[N-1-n] = u[2n+1];  C[k] = Re(exp(-i pi k/(2N)) V[k]),
// and, inversely, V[k] = exp(i pi k/(2N)) (C[k] - i C[N-k]) (C[N] = 0),
// v = IFFT(V), u[2n] = v[n], u[2n+1] = v[N-1-n].
// The FFT runs in LDS: radix-2 decimation in time, in place, the input
// placed at bit-reversed positions as it is loaded.  Twiddles are FP64
// values rounded once to fp32, from a host table.
//
// A workgroup transforms LB lines (LB/2 complex pairs) and writes each
// output line as one contiguous row.  Input lines are either rows of the
// input array (ROW) or its columns (COL: each row of the array contributes
// LB consecutive values), so a COL transform also transposes.  Steps of the
// plane pipeline:
//   forward 1: COL over the frame X[y][x] along y      -> F1[x][ky]
//   forward 2: COL over F1 along x                     -> F[ky][kx]
//   inverse 1: ROW over F along kx, scaled by H_y[ky] H_x[kx] / (N_y N_x)
//                                                      -> G[ky][x]
//   inverse 2: COL over G along ky                     -> L[x][y]
// which leaves L in the transposed layout of the direct blur's planes.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "dct.h"

namespace dog {

namespace {

constexpr int kNT = 256;

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

// In-place FFT of P lines of N complex values in LDS (input at bit-reversed
// positions, output in natural order): the radix-2 decimation-in-time
// stages, taken two at a time from registers (each thread loads four
// elements i, i+h, i+2h, i+3h of a block of 4h, applies stage s to the pairs
// (i, i+h), (i+2h, i+3h) and stage s+1 to (i, i+2h), (i+h, i+3h), and
// stores them), then a last single stage when log2 N is odd.  tw[t] =
// exp(-2 pi i t / N); INV conjugates the twiddles (no 1/N).
template <bool INV>
__device__ __forceinline__ float2 twid(const float2* tw, uint32_t t)
{
    float2 w = tw[t];
    if (INV)
        w.y = -w.y;
    return w;
}

template <bool INV>
__device__ __forceinline__ void bfly(float2& a, float2& b, float2 w)
{
    const float2 t = cmul(w, b);
    b = make_float2(a.x - t.x, a.y - t.y);
    a = make_float2(a.x + t.x, a.y + t.y);
}

template <bool INV>
__device__ void fft_lines(float2* buf, const float2* tw, int logp, int logn)
{
    const uint32_t groups = 1u << (logp + logn - 2);   // blocks of 4 elements, all lines
    int s = 0;
    for (; s + 1 < logn; s += 2) {
        const uint32_t h = 1u << s;
        for (uint32_t g = threadIdx.x; g < groups; g += kNT) {
            const uint32_t p = g >> (logn - 2);
            const uint32_t j = g & ((1u << (logn - 2)) - 1u);
            const uint32_t q = j & (h - 1u);
            const uint32_t i0 = (p << logn) + ((j >> s) << (s + 2)) + q;
            float2 a0 = buf[i0], a1 = buf[i0 + h], a2 = buf[i0 + 2 * h], a3 = buf[i0 + 3 * h];
            const float2 w1 = twid<INV>(tw, q << (logn - s - 1));
            bfly<INV>(a0, a1, w1);
            bfly<INV>(a2, a3, w1);
            bfly<INV>(a0, a2, twid<INV>(tw, q << (logn - s - 2)));
            bfly<INV>(a1, a3, twid<INV>(tw, (q + h) << (logn - s - 2)));
            buf[i0] = a0;
            buf[i0 + h] = a1;
            buf[i0 + 2 * h] = a2;
            buf[i0 + 3 * h] = a3;
        }
        __syncthreads();
    }
    if (s < logn) {   // the last stage on its own: pairs (q, q + N/2)
        const uint32_t half = 1u << (logn - 1);
        for (uint32_t g = threadIdx.x; g < (groups << 1); g += kNT) {
            const uint32_t p = g >> (logn - 1);
            const uint32_t q = g & (half - 1u);
            const uint32_t i0 = (p << logn) + q;
            float2 a = buf[i0], b = buf[i0 + half];
            bfly<INV>(a, b, twid<INV>(tw, q));
            buf[i0] = a;
            buf[i0 + half] = b;
        }
        __syncthreads();
    }
}

}  // namespace

// Elements per thread of the load and store phases are at most kE (lines
// per job are chosen so that (lines / 2) * N <= kE * kNT); those loops are
// unrolled so every thread issues all its global loads before it waits.
constexpr int kE = 16;

// One workgroup per job.  Dynamic LDS: lines/2 sequences of N float2, then
// N/2 twiddles.
template <bool INV>
__global__ void __launch_bounds__(kNT) k_dct(LaunchArgs a, const DctJob* jobs)
{
    extern __shared__ __align__(16) float2 lds[];
    DctJob J = jobs[blockIdx.x];
    if (!J.in) {
        // the frame's own pixels (their pointer changes between launches of
        // the same tables; the descriptor carries it)
        const FrameDesc& f = a.frames ? a.frames[J.frame] : a.f0;
        J.in = f.src;
        J.in_pitch = (int32_t)f.src_stride;
    }
    const uint32_t N = (uint32_t)J.N;
    const int logn = J.logn;
    const int logp = J.logp;             // log2 of the pairs of lines
    const uint32_t P = 1u << logp;
    const uint32_t total = P << logn;    // complex elements of the job
    float2* buf = lds;
    float2* tw = lds + total;
    for (uint32_t t = threadIdx.x; t < N / 2; t += kNT)
        tw[t] = J.tw[t];
    const uint32_t tid = threadIdx.x;
    const float* in = J.in;
    const size_t pitch = (size_t)J.in_pitch;
    // element e: pair p and position n; COL: the P pairs of a row are
    // consecutive (the row's 2P values), ROW: the positions of a line are
    const auto split = [&](uint32_t e, uint32_t& p, uint32_t& n) {
        if (J.cols) {
            p = e & (P - 1u);
            n = e >> logp;
        } else {
            p = e >> logn;
            n = e & (N - 1u);
        }
    };
    // the two lines of pair p at position n
    const auto load2 = [&](uint32_t p, uint32_t n) -> float2 {
        const uint32_t l = (uint32_t)J.line0 + 2u * p;
        if (J.cols)
            return make_float2(in[(size_t)n * pitch + l], in[(size_t)n * pitch + l + 1]);
        return make_float2(in[(size_t)l * pitch + n], in[(size_t)(l + 1) * pitch + n]);
    };

    if (!INV) {
        // forward: pair p holds lines 2p (real part) and 2p+1 (imaginary);
        // the value at position n goes to bitrev(reorder(n))
        float2 v[kE];
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t e = tid + (uint32_t)q * kNT;
            uint32_t p, n;
            split(e, p, n);
            if (e < total)
                v[q] = load2(p, n);
        }
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t e = tid + (uint32_t)q * kNT;
            uint32_t p, n;
            split(e, p, n);
            if (e < total)
                buf[(p << logn) + bitrev(reorder(n, N), logn)] = v[q];
        }
    } else {
        // inverse: V[k] = exp(i pi k / (2N)) (C[k] - i C[N-k]) per line, the
        // two lines of a pair as real and imaginary parts of one sequence
        float2 c[kE], d[kE];
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t e = tid + (uint32_t)q * kNT;
            uint32_t p, k;
            split(e, p, k);
            if (e < total) {
                c[q] = load2(p, k);
                d[q] = k ? load2(p, N - k) : make_float2(0.0f, 0.0f);
            }
        }
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t e = tid + (uint32_t)q * kNT;
            uint32_t p, k;
            split(e, p, k);
            if (e < total) {
                float2 cc = c[q], dd = d[q];
                const uint32_t km = (N - k) & (N - 1u);
                if (J.hline) {
                    const uint32_t l = (uint32_t)J.line0 + 2u * p;
                    const float h1 = J.hline[l], h2 = J.hline[l + 1];
                    const float hk = J.hpos[k], hkm = J.hpos[km];
                    cc = make_float2(cc.x * (h1 * hk), cc.y * (h2 * hk));
                    dd = make_float2(dd.x * (h1 * hkm), dd.y * (h2 * hkm));
                }
                const float2 e2 = J.post[k];            // exp(-i pi k / (2N))
                const float cs = e2.x, sn = -e2.y;
                const float2 V1 = make_float2(cs * cc.x + sn * dd.x, sn * cc.x - cs * dd.x);
                const float2 V2 = make_float2(cs * cc.y + sn * dd.y, sn * cc.y - cs * dd.y);
                buf[(p << logn) + bitrev(k, logn)] = make_float2(V1.x - V2.y, V1.y + V2.x);
            }
        }
    }
    __syncthreads();
    fft_lines<INV>(buf, tw, logp, logn);

    // ---- store: line l of the output is one contiguous row
    if (!INV) {
#pragma unroll
        for (int q = 0; q < kE; ++q) {
            const uint32_t e = tid + (uint32_t)q * kNT;
            if (e < total) {
                const uint32_t p = e >> logn, k = e & (N - 1u);
                const float2 z = buf[(p << logn) + k];
                const float2 zm = buf[(p << logn) + ((N - k) & (N - 1u))];
                // V1 = (Z[k] + conj Z[-k]) / 2, V2 = (Z[k] - conj Z[-k]) / (2i)
                const float2 V1 = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
                const float2 V2 = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));
                const float2 e2 = J.post[k];   // exp(-i pi k / (2N))
                const uint32_t l = (uint32_t)J.line0 + 2u * p;
                J.out[(size_t)l * J.out_pitch + k] = e2.x * V1.x - e2.y * V1.y;
                J.out[(size_t)(l + 1) * J.out_pitch + k] = e2.x * V2.x - e2.y * V2.y;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < kE / 2; ++q) {
            const uint32_t e = tid + (uint32_t)q * kNT;
            if (e < total / 2) {
                const uint32_t p = e >> (logn - 1), n = e & ((N >> 1) - 1u);
                const float2 x = buf[(p << logn) + n];            // v[n]     -> u[2n]
                const float2 y = buf[(p << logn) + N - 1u - n];   // v[N-1-n] -> u[2n+1]
                const uint32_t l = (uint32_t)J.line0 + 2u * p;
                *reinterpret_cast<float2*>(J.out + (size_t)l * J.out_pitch + 2 * n) =
                    make_float2(x.x, y.x);
                *reinterpret_cast<float2*>(J.out + (size_t)(l + 1) * J.out_pitch + 2 * n) =
                    make_float2(x.y, y.y);
            }
        }
    }
}

}  // namespace dog

extern "C" {

size_t dogk_dct_lds_bytes(int N, int lines)
{
    return ((size_t)(lines / 2) * (size_t)N + (size_t)N / 2) * sizeof(float2);
}

hipError_t dogk_dct(const dog::LaunchArgs* args, const dog::DctJob* d_jobs, int n_jobs,
                    size_t lds_bytes, int inverse, hipStream_t stream, hipEvent_t* ev)
{
    if (n_jobs <= 0)
        return hipSuccess;
    const size_t lds = lds_bytes;
    const void* fn = inverse ? reinterpret_cast<const void*>(&dog::k_dct<true>)
                             : reinterpret_cast<const void*>(&dog::k_dct<false>);
    static size_t allowed[2] = {0, 0};   // dynamic LDS each kernel has been allowed
    if (lds > allowed[inverse ? 1 : 0]) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess)
            return e;
        allowed[inverse ? 1 : 0] = lds;
    }
    const dog::DctJob* jobs = d_jobs;
    void* params[] = {const_cast<dog::LaunchArgs*>(args), &jobs};
    return ev ? hipExtLaunchKernel(fn, dim3(n_jobs), dim3(dog::kNT), params, lds, stream, ev[0],
                                   ev[1], 0)
              : hipLaunchKernel(fn, dim3(n_jobs), dim3(dog::kNT), params, lds, stream);
}

}  // extern "C"
