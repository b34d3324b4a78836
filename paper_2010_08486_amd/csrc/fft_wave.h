// Transform-domain job run by one wavefront (device code), for lines of 512,
// 1024 and 2048 values; shared by the transform kernel of dct.hip and the blur
// kernels of kernels.hip.  Not part of the public C ABI.
//
// The job computes what fft_job.h computes (two lines u1, u2 blurred by the
// kernels of its planes as products in the type-II cosine transform domain;
// the module comment of dct.hip gives the transforms), with the complex FFT
// of length N = 64 E laid out over the 64 lanes of one wavefront, E values
// per lane, and factored as N = E x A x B with A B = 64 (E = 32: 32 x 16 x 4;
// E = 16: 16 x 16 x 4; E = 8: 8 x 8 x 8):
//   pass 1: lane l holds x[l + 64 m], m < E, and takes the E-point DFT over m
//           in registers, then multiplies by W_N^(l k1);
//   pass 2: after an exchange through the wave's LDS buffer, each lane takes
//           E / A A-point DFTs (over n2 = B a + b for one (k1, b)), then
//           multiplies by W_64^(b c);
//   pass 3: after a second exchange, E / B B-point DFTs over b, which leave
//           X[k] for k = l (mod 64) in lane l.
// The inverse transform uses the same passes with conjugate factors, so its
// input is expected, and its output left, in that same layout.  The cosine
// coefficients need X[k] beside X[N - k]: lane l's partner is lane
// (64 - l) mod 64, reached with ds_bpermute.  Every exchange moves one
// component at a time through a buffer of WaveGeom::BUF floats, padded so
// that neither the writes nor the reads of a wave meet a bank twice; the
// wave is its only user, so wave-level ordering (no workgroup barrier)
// suffices.  The per-lane twiddle factors are FP64 values rounded once to
// fp32, from host tables laid out lane-contiguous.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dct.h"
#include "dog_internal.h"
#include "fft_job.h"

namespace dog {

// Factors and buffer sizes of a wave job with lines of 2^LOGN values.
template <int LOGN>
struct WaveGeom {
    static_assert(fft_wave_len(LOGN), "wave jobs take lines of 512, 1024 or 2048 values");
    static constexpr int N = 1 << LOGN;
    static constexpr int E = N / 64;                  // values per lane
    static constexpr int A = E >= 16 ? 16 : 8;        // pass-2 points
    static constexpr int B = 64 / A;                  // pass-3 points
    static constexpr int G2 = E / A;                  // pass-2 DFTs per lane
    static constexpr int G3 = E / B;                  // pass-3 DFTs per lane
    static constexpr int P1 = B;                      // exchange-1 row padding
    static constexpr int P2 = E >= 16 ? 8 : 4;        // exchange-2 row padding
    static constexpr int X1 = E * (64 + P1);
    static constexpr int X2 = B * (E * A + P2);
    static constexpr int BUF = X1 > X2 ? X1 : X2;     // floats per wave
    static constexpr size_t LDS_BYTES = (size_t)kFftWaveJobs * BUF * sizeof(float);
};

namespace wfft {

// cos and sin of 2 pi e / 32, e = 0..15 (the 32nd roots of unity)
constexpr float kCos32[16] = {1.0f,
                              0.98078528040323043f,    // cos(pi / 16)
                              0.92387953251128674f,    // cos(pi / 8)
                              0.83146961230254524f,    // cos(3 pi / 16)
                              0.70710678118654752f,    // cos(pi / 4)
                              0.55557023301960218f,    // cos(5 pi / 16)
                              0.38268343236508977f,    // cos(3 pi / 8)
                              0.19509032201612825f,    // cos(7 pi / 16)
                              0.0f,
                              -0.19509032201612825f,
                              -0.38268343236508977f,
                              -0.55557023301960218f,
                              -0.70710678118654752f,
                              -0.83146961230254524f,
                              -0.92387953251128674f,
                              -0.98078528040323043f};
constexpr float kSin32[16] = {0.0f,
                              0.19509032201612825f,
                              0.38268343236508977f,
                              0.55557023301960218f,
                              0.70710678118654752f,
                              0.83146961230254524f,
                              0.92387953251128674f,
                              0.98078528040323043f,
                              1.0f,
                              0.98078528040323043f,
                              0.92387953251128674f,
                              0.83146961230254524f,
                              0.70710678118654752f,
                              0.55557023301960218f,
                              0.38268343236508977f,
                              0.19509032201612825f};

constexpr int bit_rev(int i, int bits)
{
    int r = 0;
    for (int b = 0; b < bits; ++b)
        r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}
constexpr int log2c(int r) { return r <= 1 ? 0 : 1 + log2c(r / 2); }

// v exp(-2 pi i e / 32) (INV: exp(+2 pi i e / 32)), e in [0, 16); e is a
// constant once the loops around the call are unrolled, so only one branch
// remains, and the factors 1 and -i (+i) are applied exactly.
template <bool INV>
__device__ __forceinline__ float2 rot32(float2 v, int e)
{
#pragma clang fp contract(on)
    if (e == 0)
        return v;
    if (e == 8)
        return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
    const float c = kCos32[e];
    const float s = INV ? kSin32[e] : -kSin32[e];   // the factor is c + i s
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
}

// R-point DFT (R = 4, 8, 16, 32) of x[0..R-1] in registers, natural order
// in and out: radix-2 decimation in time over a bit-reversed copy.
template <int R, bool INV>
__device__ __forceinline__ void dft(float2* x)
{
#pragma clang fp contract(on)
    constexpr int LB = log2c(R);
    float2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i)
        t[bit_rev(i, LB)] = x[i];
#pragma unroll
    for (int len = 2; len <= R; len *= 2) {
#pragma unroll
        for (int i = 0; i < R; i += len) {
#pragma unroll
            for (int j = 0; j < len / 2; ++j) {
                const float2 u = t[i + j];
                const float2 v = rot32<INV>(t[i + j + len / 2], j * (32 / len));
                t[i + j] = make_float2(u.x + v.x, u.y + v.y);
                t[i + j + len / 2] = make_float2(u.x - v.x, u.y - v.y);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
        x[i] = t[i];
}

// Orders the wave's LDS accesses before and after it (the wave's LDS
// instructions execute in program order; this keeps the compiler from
// moving them across).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Multiply-adds in this file are fused only within one expression (clang fp
// contract on), so every kernel that inlines a job rounds alike: a frame's
// planes are bitwise the same whichever launch runs its jobs.

// A wave-uniform value the compiler cannot see through: loads addressed
// from it stay where they are written (inside a loop, rather than hoisted out
// of it and held in registers across the loop).
__device__ __forceinline__ uint32_t opaque(uint32_t v)
{
    v = __builtin_amdgcn_readfirstlane(v);
    asm volatile("" : "+s"(v));
    return v;
}
template <class T>
__device__ __forceinline__ T* opaque(T* p)
{
    const unsigned long long b = (unsigned long long)p;
    const uint32_t lo = opaque((uint32_t)b), hi = opaque((uint32_t)(b >> 32));
    return (T*)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ float bperm(int addr, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// v[k] *= w^k for k = 1..R-1 (R = 4, 8, 16, 32), the lane's w^(2^i) read
// from row i of t (64 lanes per row); every other power is a product of at
// most log2 R - 1 of them.  INV conjugates the factors.
template <int R, bool INV>
__device__ __forceinline__ void apply_powers(float2* v, const DOG_GLOBAL_AS float2* t, uint32_t l)
{
#pragma clang fp contract(on)
    constexpr int LB = log2c(R);
    float2 p[LB];
#pragma unroll
    for (int i = 0; i < LB; ++i) {
        p[i] = t[i * 64 + l];
        if (INV)
            p[i].y = -p[i].y;
    }
    float2 w[R];
#pragma unroll
    for (int k = 1; k < R; ++k) {
        const int hb = 31 - __builtin_clz(k);   // k = 2^hb + rest
        const int rest = k - (1 << hb);
        w[k] = rest ? fftd::cmul(p[hb], w[rest]) : p[hb];
        v[k] = fftd::cmul(v[k], w[k]);
    }
}

// In-register FFT of the wave's sequence (see the file comment).  Lane l:
// x[m] = input element l + 64 m on entry, X[l + 64 j] in x[j] on return.
// t1: log2 E rows of 64 factors W_N^(l 2^i); t2: log2 A rows of 64 factors
// W_64^((l mod B) 2^i).  INV conjugates every factor.
template <int LOGN, bool INV>
__device__ __forceinline__ void fft_wave(float2 (&x)[WaveGeom<LOGN>::E], float* buf,
                                         const DOG_GLOBAL_AS float2* t1,
                                         const DOG_GLOBAL_AS float2* t2, uint32_t l)
{
#pragma clang fp contract(on)
    using G = WaveGeom<LOGN>;
    constexpr int E = G::E, A = G::A, B = G::B, G2 = G::G2, G3 = G::G3;
    constexpr int R1 = 64 + G::P1, R2 = E * A + G::P2;
    t1 = opaque(t1);   // the factors are loaded per transform
    t2 = opaque(t2);

    // ---- pass 1: E-point DFT over m, then W_N^(l k1)
    dft<E, INV>(x);
    apply_powers<E, INV>(x, t1, l);

    // ---- exchange 1: Y[n2][k1] at k1 R1 + n2; lane l then takes
    // (k1, b) = (l / B + A g2, l mod B) and reads n2 = B a + b, a < A
    const uint32_t q = l / B, b = l % B;
    float2 y[G2][A];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        wave_sync();
#pragma unroll
        for (int k = 0; k < E; ++k)
            buf[k * R1 + l] = comp ? x[k].y : x[k].x;
        wave_sync();
#pragma unroll
        for (int g = 0; g < G2; ++g)
#pragma unroll
            for (int a = 0; a < A; ++a) {
                const float v = buf[(q + A * g) * R1 + B * a + b];
                if (comp)
                    y[g][a].y = v;
                else
                    y[g][a].x = v;
            }
    }

    // ---- pass 2: A-point DFTs over a, then W_64^(b c)
#pragma unroll
    for (int g = 0; g < G2; ++g) {
        dft<A, INV>(y[g]);
        apply_powers<A, INV>(y[g], t2, l);
    }

    // ---- exchange 2: Z[k1][b][c] at b R2 + k1 + E c; lane l then takes the
    // (k1, c) with k1 + E c = l + 64 g3 and reads b' < B
    float2 z[G3][B];
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        wave_sync();
#pragma unroll
        for (int g = 0; g < G2; ++g)
#pragma unroll
            for (int c = 0; c < A; ++c)
                buf[b * R2 + q + A * g + E * c] = comp ? y[g][c].y : y[g][c].x;
        wave_sync();
#pragma unroll
        for (int g = 0; g < G3; ++g)
#pragma unroll
            for (int bb = 0; bb < B; ++bb) {
                const float v = buf[bb * R2 + l + 64 * g];
                if (comp)
                    z[g][bb].y = v;
                else
                    z[g][bb].x = v;
            }
    }

    // ---- pass 3: B-point DFTs over b: X[l + 64 (g3 + G3 d)]
#pragma unroll
    for (int g = 0; g < G3; ++g) {
        dft<B, INV>(z[g]);
#pragma unroll
        for (int d = 0; d < B; ++d)
            x[g + G3 * d] = z[g][d];
    }
}

}  // namespace wfft

// The job at jp, run by one wavefront with its own `buf` (WaveGeom::BUF
// floats of LDS): one plane (a job with no planes is padding and returns at
// once).  VEC: the input's pairs of values (a row job's u[2n], u[2n+1]; a
// column job's two lines) are 8-byte aligned.  PRE: x already holds the
// job's lines in the layout fft_wave takes (fft_wave_load_cols); else the
// job loads them into x.  jp->post is followed by the
// factor tables of fft_wave: log2 E rows of 64, then log2 A rows of 64.
template <int LOGN, bool VEC, bool PRE = false>
__device__ __forceinline__ void fft_wave_job(const LaunchArgs& a, const FftJob* __restrict__ jp,
                                             float* buf, float2 (&x)[WaveGeom<LOGN>::E])
{
#pragma clang fp contract(on)
    using namespace fftd;
    using G = WaveGeom<LOGN>;
    constexpr uint32_t N = G::N, half = N / 2;
    constexpr int E = G::E;
    static_assert(kFftLines == 2, "one complex sequence per job");
    if (!PRE && jp->n_planes <= 0)   // (a group loaded together has no padding)
        return;
    const float* in = jp->in;
    long long pitch = jp->in_pitch;
    if (!in) {
        const FrameDesc& f = a.frames ? a.frames[jp->frame] : a.f0;
        in = f.src;
        pitch = f.src_stride;
    }
    const uint32_t line0 = (uint32_t)jp->line0;
    const bool in_rows = jp->in_rows != 0;
    const uint32_t out_pitch = (uint32_t)jp->out_pitch;
    const auto post_g = gptr(jp->post);
    const auto t1 = post_g + N;
    const auto t2 = t1 + wfft::log2c(E) * 64;
    const auto out = gptr_w(jp->planes->out[0]);
    const auto hg = gptr(jp->planes->h[0]);
    const uint32_t l = threadIdx.x & 63u;

    // ---- the lines as z = v1 + i v2, v the even/odd reordering of u:
    // element n = l + 64 m is u[2n] below N/2, u[2N - 1 - 2n] above.  Rows:
    // lane l reads the pair u[2n], u[2n+1] of each line for n = l + 64 m,
    // m < E/2 (consecutive lanes, consecutive pairs); u[2n+1] is element
    // N - 1 - n, which lane 63 - l holds (index E - 1 - m).
    const int mirror = (int)((63u - l) << 2);
    const auto in_g = gptr(in);
    if (PRE) {
        // x already holds the lines (fft_wave_load_cols)
    } else if (in_rows) {
        const auto r1 = in_g + (size_t)line0 * pitch;
        const auto r2 = r1 + pitch;
        float2 p1[E / 2], p2[E / 2];
#pragma unroll
        for (int m = 0; m < E / 2; ++m) {
            const uint32_t o = 2u * (l + 64u * m);
            if (VEC) {
                p1[m] = *reinterpret_cast<const DOG_GLOBAL_AS float2*>(r1 + o);
                p2[m] = *reinterpret_cast<const DOG_GLOBAL_AS float2*>(r2 + o);
            } else {
                p1[m] = make_float2(r1[o], r1[o + 1]);
                p2[m] = make_float2(r2[o], r2[o + 1]);
            }
        }
#pragma unroll
        for (int m = 0; m < E / 2; ++m) {
            x[m] = make_float2(p1[m].x, p2[m].x);
            x[E - 1 - m] = make_float2(wfft::bperm(mirror, p1[m].y), wfft::bperm(mirror, p2[m].y));
        }
    } else {
        // (32-bit offsets: a column job's input is a plane of at most
        // 2048 x 2048 values)
        const uint32_t pt = (uint32_t)pitch;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const uint32_t n = l + 64u * m;
            const uint32_t r = n < half ? 2u * n : 2u * N - 1u - 2u * n;
            const uint32_t o = r * pt + line0;
            if (VEC)
                x[m] = *reinterpret_cast<const DOG_GLOBAL_AS float2*>(in_g + o);
            else
                x[m] = make_float2(in_g[o], in_g[o + 1]);
        }
    }
    // exp(-i pi k / (2N)) at k = l + 64 j is post[l] post[64 j]; the second
    // factor is the same for every lane (scalar loads)
    const float2 el = post_g[l];
    const auto post_c = (const DOG_CONST_AS float2*)(jp->post);
    wfft::fft_wave<LOGN, false>(x, buf, t1, t2, l);
    // the transfer function H[k] / N at k = l + 64 j
    float hk[E];
#pragma unroll
    for (int j = 0; j < E; ++j)
        hk[j] = hg[l + 64u * j];

    // ---- P[k] = H_k C_k per line, C[k] = Re(exp(-i pi k / (2N)) V[k]) the
    // cosine coefficients, V1 = (Z[k] + conj Z[N-k]) / 2, V2 = (Z[k] -
    // conj Z[N-k]) / (2i): Z[N - k] from the partner lane (lane 0 holds both
    // k = 64 j and N - k = 64 (E - j) itself)
    const int partner = (int)(((64u - l) & 63u) << 2);
    float p1[E], p2[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const float2 z = x[j];
        float2 zm = make_float2(wfft::bperm(partner, x[E - 1 - j].x),
                                wfft::bperm(partner, x[E - 1 - j].y));
        if (l == 0)
            zm = x[(E - j) % E];
        const float2 V1 = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
        const float2 V2 = make_float2(0.5f * (z.y + zm.y), 0.5f * (zm.x - z.x));
        const float2 e = cmul(el, post_c[64 * j]);   // (cos, -sin) of pi k / (2N)
        p1[j] = hk[j] * (e.x * V1.x - e.y * V1.y);
        p2[j] = hk[j] * (e.x * V2.x - e.y * V2.y);
        if (j % 4 == 3)
            __builtin_amdgcn_sched_barrier(0);   // bounds the values in flight
    }

    // ---- inverse sequence V[k] = exp(i pi k / (2N)) (P_k - i P_{N-k}),
    // P_N = 0; P_{N-k} from the partner lane (lane 0: its own P at 64 (E - j))
#pragma unroll
    for (int j = 0; j < E; ++j) {
        float b1 = wfft::bperm(partner, p1[E - 1 - j]);
        float b2 = wfft::bperm(partner, p2[E - 1 - j]);
        if (l == 0) {
            b1 = j ? p1[E - j] : 0.0f;
            b2 = j ? p2[E - j] : 0.0f;
        }
        const float2 e = cmul(el, post_c[64 * j]);
        const float c = e.x, s = -e.y;
        const float2 V1 = make_float2(c * p1[j] + s * b1, s * p1[j] - c * b1);
        const float2 V2 = make_float2(c * p2[j] + s * b2, s * p2[j] - c * b2);
        x[j] = make_float2(V1.x - V2.y, V1.y + V2.x);
        if (j % 4 == 3)
            __builtin_amdgcn_sched_barrier(0);
    }
    wfft::fft_wave<LOGN, true>(x, buf, t1, t2, l);

    // ---- store: u[2n] = v[n], u[2n+1] = v[N-1-n] per line, the lines rows
    // line0 and line0 + 1 of the plane: lane l writes the pairs at
    // n = l + 64 j, j < E/2 (v[N-1-n] from lane 63 - l, index E - 1 - j)
    auto row1 = out + (size_t)line0 * out_pitch;
    auto row2 = row1 + out_pitch;
#pragma unroll
    for (int j = 0; j < E / 2; ++j) {
        const float ox = wfft::bperm(mirror, x[E - 1 - j].x);
        const float oy = wfft::bperm(mirror, x[E - 1 - j].y);
        const uint32_t o = 2u * (l + 64u * j);
        *reinterpret_cast<DOG_GLOBAL_AS float2*>(row1 + o) = make_float2(x[j].x, ox);
        *reinterpret_cast<DOG_GLOBAL_AS float2*>(row2 + o) = make_float2(x[j].y, oy);
    }
}

// Loads the lines of the four column jobs at g (marked kFftGroupCols) for
// the four wavefronts of a workgroup of 256 threads, wave w taking lines
// line0 + 2w, + 2w + 1: chunks of 256 input rows, each row's 8 values read
// with two 16-byte loads (32 rows per load instruction, where the waves'
// own 8-byte loads would touch 64) into the workgroup's LDS (rows padded to
// 9 floats), then each wave's elements of the chunk from there.  Every
// thread of the workgroup calls it (workgroup barriers); `lds` holds
// 256 x 9 floats; x receives what fft_wave_job's own column loads would.
template <int LOGN>
__device__ __forceinline__ void fft_wave_load_cols(const FftJob* __restrict__ g, float* lds,
                                                   float2 (&x)[WaveGeom<LOGN>::E])
{
    constexpr uint32_t N = 1u << LOGN, half = N / 2;
    constexpr int E = WaveGeom<LOGN>::E, CH = 256, RS = 9;
    static_assert(CH * RS <= kFftWaveJobs * WaveGeom<LOGN>::BUF, "chunk fits the wave buffers");
    const auto in = fftd::gptr(g->in);
    const uint32_t pitch = (uint32_t)g->in_pitch, col0 = (uint32_t)g->line0;
    const uint32_t t = threadIdx.x, w = t >> 6, l = t & 63u;
    const uint32_t tr = t >> 1, th = (t & 1u) * 4u;
#pragma unroll
    for (int c = 0; c < (int)N / CH; ++c) {
        float4 v[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            v[i] = *reinterpret_cast<const DOG_GLOBAL_AS float4*>(
                in + (c * CH + tr + 128u * i) * pitch + col0 + th);
        if (c > 0)
            __syncthreads();   // the previous chunk's reads are done
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float* d = lds + (tr + 128u * i) * RS + th;
            d[0] = v[i].x;
            d[1] = v[i].y;
            d[2] = v[i].z;
            d[3] = v[i].w;
        }
        __syncthreads();
        // this chunk's elements: m = 2c, 2c + 1 (rows 2n) and E - 2 - 2c,
        // E - 1 - 2c (rows 2N - 1 - 2n)
        const int ms[4] = {2 * c, 2 * c + 1, E - 2 - 2 * c, E - 1 - 2 * c};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t n = l + 64u * ms[q];
            const uint32_t r = n < half ? 2u * n : 2u * N - 1u - 2u * n;
            const float* s = lds + (r - c * CH) * RS + 2u * w;
            x[ms[q]] = make_float2(s[0], s[1]);
        }
        // the chunk's values in registers before the next barrier: a read
        // left behind it (the compiler may sink loads past s_barrier, which
        // it does not count as a memory operation) would race with the
        // next chunk's writes or with another wave's exchanges
#pragma unroll
        for (int q = 0; q < 4; ++q)
            asm volatile("" : "+v"(x[ms[q]].x), "+v"(x[ms[q]].y));
    }
    __syncthreads();   // the buffers are the waves' own again
}

// LDS bytes a workgroup of NW wavefronts needs to run the jobs of lines of
// 2^LOGN values inside a blur launch (the largest size_t: it cannot).
template <int LOGN, int NW>
constexpr size_t fft_merged_lds()
{
    if constexpr (fft_wave_len(LOGN))
        return NW >= kFftWaveJobs ? WaveGeom<LOGN>::LDS_BYTES : ~(size_t)0;
    else
        return FftGeom<LOGN, 64 * NW>::LDS_BYTES;
}

}  // namespace dog
