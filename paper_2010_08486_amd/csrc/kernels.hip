// HIP kernels (gfx950) of the Difference-of-Gaussians detector hot path.
//
//   pass 1  : Gaussian blur down the columns of the input frame, one plane of
//             the sigma ladder per work unit, written transposed (Sec. 3 scale
//             space, Sec. 4.1 truncated kernels).
//   pass 2  : the same blur down the columns of the transposed pass-1 plane,
//             i.e. along the rows of the original frame; the result L_p stays
//             in the transposed layout.
//   nms     : DoG D_i = sigma_i (L_i - L_{i+1}) formed in registers (Sec. 4
//             Eq. 2-3), 3x3x3 maximum over (x, y, scale) with out-of-cube
//             neighbours ignored, equality test and strict threshold (Sec. 4
//             local-maximum heuristic, Sec. 4.1 Thresh mask), and wavefront
//             ballot compaction of the survivors into a record list.
//
// The blur is a direct truncated stencil, not a dense contraction, so it runs
// on the FP32 vector ALUs: each lane owns one column and S consecutive outputs
// along the walking direction, streams its input column once per tap chunk,
// and takes the (wave-uniform) weights from scalar registers, so each loaded
// value feeds S fused multiply-adds.  A ring of R row buffers keeps R-1 chunks
// of loads in flight ahead of the multiply-adds.  Reflection at the borders
// only ever applies to the walking direction, where the row index is uniform,
// so the interior path has no per-lane boundary logic at all.
//
// Each kernel runs one workgroup per tile and reads its tile from a host-built
// table: widest kernels first (the dispatcher hands out workgroups in order,
// which balances the uneven tap counts), with XCD-local column slices
// interleaved so workgroup b, placed on XCD b mod 8, stays in that XCD's L2.
// No atomics are needed to distribute work.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "dog_internal.h"
#include "fft_job.h"
#include "fft_wave.h"

// Pointers into the constant (scalar-load) address space.  The qualifier only
// exists for the device compilation pass; the host pass of this file sees
// plain pointers.
#if defined(__HIP_DEVICE_COMPILE__)
#define DOG_CONSTANT_AS __attribute__((address_space(4)))
#else
#define DOG_CONSTANT_AS
#endif

namespace dog {

// Scalar view of the launch tables: they are read-only during a launch and
// indexed uniformly, so their fields land in scalar registers.
template <class T>
__device__ __forceinline__ const DOG_CONSTANT_AS T* cst(const T* p)
{
    return (const DOG_CONSTANT_AS T*)p;
}

typedef const DOG_CONSTANT_AS float* cptr_t;

// Buffer resource over one plane: raw (unswizzled) dword loads with a scalar
// row offset and a per-lane column offset; the hardware range check returns 0
// for any byte offset at or beyond `bytes` instead of touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

__device__ __forceinline__ float load_f32(__amdgpu_buffer_rsrc_t rs, unsigned voff, int soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, soff, 0));
}

// v[m] = column voff/4 of row refl(row0 + m), m = 0..S-1.  The byte offset of
// every (reflected) row comes from a per-frame table read with scalar loads,
// so interior and border strips run the same code and each lane keeps a
// single column offset.
template <int S>
__device__ __forceinline__ void load_rows(float (&v)[S], __amdgpu_buffer_rsrc_t rs, unsigned voff,
                                          const DOG_CONSTANT_AS int* rows, int row0)
{
#pragma unroll
    for (int m = 0; m < S; ++m)
        v[m] = load_f32(rs, voff, rows[row0 + m]);
}

// One chunk of S taps: acc[t] += sum_u wc[u] * window[u + t], where the
// window is lo[0..S-1] followed by hi[0..S-1].
template <int S>
__device__ __forceinline__ void fma_chunk(float (&acc)[S], const float (&lo)[S],
                                          const float (&hi)[S], cptr_t wc)
{
#pragma unroll
    for (int u = 0; u < S; ++u) {
        const float wu = wc[u];
#pragma unroll
        for (int t = 0; t < S; ++t)
            acc[t] = __builtin_fmaf(wu, (u + t < S) ? lo[u + t] : hi[u + t - S], acc[t]);
    }
}

// nch chunks of S taps.  Chunk ch multiplies row chunks X_ch and X_{ch+1}
// (X_j = rows base + j*S .. base + j*S + S - 1).  The ring X[0..R-1] holds
// X_ch .. X_{ch+R-2} when chunk ch starts and the load of X_{ch+R-1} is issued
// before its multiply-adds, so R-1 chunks of loads are in flight.
// Reads table rows up to base + (nch + R - 1) * S - 1.
template <int S, int R>
__device__ __forceinline__ void blur_chunks(__amdgpu_buffer_rsrc_t rs, unsigned voff,
                                            const DOG_CONSTANT_AS int* rows, int base, int nch,
                                            cptr_t w, float (&acc)[S])
{
    float X[R][S];
#pragma unroll
    for (int j = 0; j < R - 1; ++j)
        load_rows<S>(X[j], rs, voff, rows, base + j * S);
    int ch = 0;
    for (; ch + R <= nch; ch += R) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            load_rows<S>(X[(q + R - 1) % R], rs, voff, rows, base + (ch + q + R - 1) * S);
            fma_chunk<S>(acc, X[q], X[(q + 1) % R], w + (ch + q) * S);
        }
    }
    // fewer than R chunks left; X[0..R-2] hold X_ch .. X_{ch+R-2}
#pragma unroll
    for (int q = 0; q < R - 1; ++q) {
        if (q < nch - ch) {
            if (q == R - 2)
                load_rows<S>(X[R - 1], rs, voff, rows, base + (ch + R - 1) * S);
            fma_chunk<S>(acc, X[q], X[q + 1], w + (ch + q) * S);
        }
    }
}

// acc[t] = sum_{j=0}^{2r} w[j] * col[refl(y0 - r + t + j)], t = 0..S-1, where
// col[m] is column c of row m of the plane behind `rs` and rows[t] is the byte
// offset of row refl(t).  Taps are accumulated in ascending order, so every
// output sees the same summation order whatever the tile shape; w must be
// zero-padded up to ceil((2r+1)/S)*S.
template <int S, int R>
__device__ __forceinline__ void blur_strip(__amdgpu_buffer_rsrc_t rs, const int* rows, int c,
                                           int y0, int r, const float* w, float (&acc)[S])
{
#pragma unroll
    for (int t = 0; t < S; ++t)
        acc[t] = 0.0f;
    blur_chunks<S, R>(rs, (unsigned)c * 4u, cst(rows), y0 - r, (2 * r + S) / S, (cptr_t)w, acc);
}

// This workgroup's tile.
__device__ __forceinline__ Tile my_tile(const Tile* table)
{
    return cst(table)[blockIdx.x];
}

// Descriptor of frame fi: from the frame table, or the one passed inline in
// the kernel arguments of a one-frame launch.
__device__ __forceinline__ FrameDesc frame_of(const LaunchArgs& a, int fi)
{
    return a.frames ? cst(a.frames)[fi] : a.f0;
}

// Pass 1: T_p = column blur of the input frame, stored transposed.
// Tile = 64 columns x (S*NW*BI) rows of one (frame, plane) unit.
template <int S, int R, int NW, int BI>
__global__ void __launch_bounds__(64 * NW) k_pass1(LaunchArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    constexpr int BAND = S * NW * BI;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        a.cand->count = 0u;  // read by the local-maximum kernel of this sequence
    {
        const Tile tl = my_tile(a.tiles1);
        const int cb = tl.cb;
        const int band = tl.band;
        const FrameDesc f = frame_of(a, tl.frame);
        const int p = tl.plane;
        const int r = cst(a.ladders)[f.ladder].r[p];
        const float* w = a.weights + cst(a.ladders)[f.ladder].woff[p];
        const int col = cb * 64 + lane;
        const __amdgpu_buffer_rsrc_t rs =
            plane_rsrc(f.src, (unsigned)(((long long)(f.H - 1) * f.src_stride + f.W) * 4));
        const int* rows = f.rows1 + f.pad;
        if (col < f.W) {
            for (int q = 0; q < BI; ++q) {
                const int y0 = band * BAND + (q * NW + wv) * S;
                if (y0 >= f.H)
                    break;
                float acc[S];
                blur_strip<S, R>(rs, rows, col, y0, r, w, acc);
                float* __restrict__ dst = f.T + ((long long)p * f.W + col) * f.pitch + y0;
                if (y0 + S <= f.H) {
#pragma unroll
                    for (int t = 0; t < S; t += 4)
                        *reinterpret_cast<float4*>(dst + t) =
                            make_float4(acc[t], acc[t + 1], acc[t + 2], acc[t + 3]);
                } else {
#pragma unroll
                    for (int t = 0; t < S; ++t)
                        if (y0 + t < f.H)
                            dst[t] = acc[t];
                }
            }
        }
    }
}

// Pass 2: L_p = blur of T_p down its columns (along x of the frame); output in
// the same transposed layout.  Tile = 64 columns (y) x (S*NW*BI) rows (x).
template <int S, int R, int NW, int BI>
__global__ void __launch_bounds__(64 * NW) k_pass2(LaunchArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    constexpr int BAND = S * NW * BI;
    {
        const Tile tl = my_tile(a.tiles2);
        const int cb = tl.cb;
        const int band = tl.band;
        const FrameDesc f = frame_of(a, tl.frame);
        const int p = tl.plane;
        const int r = cst(a.ladders)[f.ladder].r[p];
        const float* w = a.weights + cst(a.ladders)[f.ladder].woff[p];
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(f.T + (long long)p * f.W * f.pitch,
                                                     (unsigned)((long long)f.W * f.pitch * 4));
        const int* rows = f.rows2 + f.pad;
        float* __restrict__ dstp = f.L + (long long)p * f.W * f.pitch;
        const int col = cb * 64 + lane;
        if (col < f.H) {
            for (int q = 0; q < BI; ++q) {
                const int x0 = band * BAND + (q * NW + wv) * S;
                if (x0 >= f.W)
                    break;
                float acc[S];
                blur_strip<S, R>(rs, rows, col, x0, r, w, acc);
#pragma unroll
                for (int t = 0; t < S; ++t)
                    if (x0 + t < f.W)
                        dstp[(long long)(x0 + t) * f.pitch + col] = acc[t];
            }
        }
    }
}

// ------------------------------------------------------------------------
// LDS-staged blur (both passes).  A workgroup of NW waves owns 64 columns and
// NW*S consecutive outputs along the blur direction; wave w computes outputs
// w*S .. w*S+S-1 of the band for its lane's column.  Input rows stream
// through an LDS ring of NW+2 chunks of S rows: each chunk is fetched from
// HBM/L2 once per workgroup with 16-byte loads (one per lane for S = 16,
// NW = 4), P chunks ahead of use, instead of once per wave with 4-byte loads.
// Step c multiplies row chunks X_{w+c} and X_{w+c+1} by taps c*S .. c*S+S-1,
// exactly as blur_chunks does, so results are bitwise identical to the
// register-ring kernels.  Weights are moved into vector registers once per
// chunk: gfx950 issues FP32 FMAs whose operands are all vector registers at
// twice the rate of the form that reads a scalar register.

// Half-sample symmetric reflection of row t into [0, n) (period 2n).
__device__ __forceinline__ int refl_row(int t, int n)
{
    if ((unsigned)t < (unsigned)n)
        return t;
    const int p = 2 * n;
    int u = t % p;
    if (u < 0)
        u += p;
    return u < n ? u : p - 1 - u;
}

__device__ __forceinline__ float to_vgpr(float s)
{
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// The same multiply-adds as fma_chunk, issued by window row m = u + t: every
// product with the register-held chunk `lo` comes before any with `hi`, so
// the LDS reads of `hi` overlap the first half.  For each output t the taps
// still arrive in ascending u, so the sums are bitwise those of fma_chunk.
template <int S>
__device__ __forceinline__ void fma_chunk_v(float (&acc)[S], const float (&lo)[S],
                                            const float (&hi)[S], const float (&wv)[S])
{
#pragma unroll
    for (int m = 0; m < 2 * S - 1; ++m) {
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const int u = m - t;
            if (u >= 0 && u < S)
                acc[t] = __builtin_fmaf(wv[u], m < S ? lo[m] : hi[m - S], acc[t]);
        }
    }
}

// Taps of one plane kept in LDS by the staged blur (larger planes read them
// with scalar loads): 512 floats cover radii up to 247.
constexpr int kLdsWeights = 512;

template <int S, int NW>
struct StageGeom {
    static constexpr int Q = NW + 2;                        // LDS ring slots
    static constexpr int NT = 64 * NW;                      // threads
    static constexpr int LPL = (16 * S + NT - 1) / NT;      // 16-byte loads per lane per chunk
};

// Fetch row chunk j (rows base + j*S .. + S-1, reflected into [0, n)) of the
// 64 columns from col0 into registers: thread q of the chunk holds columns
// col0 + 4*(q%16) .. +3 of row q/16.  WIDE: every 64-column block lies inside
// the rows and rows are 16-byte aligned, so one 16-byte load per thread; else
// four 4-byte loads, which the buffer range check turns into zeros past the
// plane (such columns are never stored).  The number of loads is fixed, so
// the compiler can wait for one staged chunk while later ones stay in flight.
template <int S, int NW, bool WIDE, int L>
__device__ __forceinline__ void stage_load(float4 (&st)[L], __amdgpu_buffer_rsrc_t rs, int tid,
                                           int base, int j, int n, int stride, int col0)
{
    using G = StageGeom<S, NW>;
    static_assert(L == G::LPL, "staging registers");
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int q = tid + i * G::NT;
        if ((16 * S) % G::NT == 0 || q < 16 * S) {
            const int row = refl_row(base + j * S + (q >> 4), n);
            const unsigned off = (unsigned)(row * stride + col0 + 4 * (q & 15)) * 4u;
            if (WIDE) {
                st[i] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
            } else {
                st[i].x = load_f32(rs, off, 0);
                st[i].y = load_f32(rs, off + 4u, 0);
                st[i].z = load_f32(rs, off + 8u, 0);
                st[i].w = load_f32(rs, off + 12u, 0);
            }
        }
    }
}

template <int S, int NW, int L>
__device__ __forceinline__ void stage_store(float4* lds, int slot, const float4 (&st)[L], int tid)
{
    using G = StageGeom<S, NW>;
    static_assert(L == G::LPL, "staging registers");
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int q = tid + i * G::NT;
        if ((16 * S) % G::NT == 0 || q < 16 * S)
            lds[slot * S * 16 + q] = st[i];
    }
}

template <int S>
__device__ __forceinline__ void lds_rows(float (&v)[S], const float* lds, int slot, int lane)
{
#pragma unroll
    for (int m = 0; m < S; ++m)
        v[m] = lds[(slot * S + m) * 64 + lane];
}

// PASS 1: blur down the columns of the input frame into T (transposed);
// PASS 2: blur down the columns of T_p into L_p (same layout).
// GROUP: a tile may take a run of planes (Tile::n_planes); else one plane
// (the plane loop costs registers).  FFTLOGN > 0: the launch also runs the
// pass's transform-domain jobs (lines of 2^FFTLOGN values, fft_job.h) in its
// first a.n_fft[PASS - 1] workgroups, with the ring's LDS, before the direct
// tiles.
template <int PASS, int S, int NW, int P, bool WIDE, int FFTLOGN = 0, bool GROUP = false>
__global__ void __launch_bounds__(64 * NW) k_blur_lds(LaunchArgs a)
{
    using G = StageGeom<S, NW>;
    static_assert(S % 4 == 0 && S <= 16 && P >= 1, "tile geometry");
    __shared__ float4 lds4[G::Q * S * 16];
    __shared__ float4 wl4[kLdsWeights / 4];
    const float* lds = reinterpret_cast<const float*>(lds4);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(tid >> 6));
    if (PASS == 1 && blockIdx.x == 0 && tid == 0)
        a.cand->count = 0u;  // read by the local-maximum kernel of this sequence
    int wg = blockIdx.x;
    if constexpr (FFTLOGN > 0) {
        static_assert(fft_merged_lds<FFTLOGN, NW>() <= sizeof(lds4), "jobs fit the ring");
        const int nf = a.n_fft[PASS - 1];
        if (wg < nf) {
            if constexpr (fft_wave_len(FFTLOGN)) {
                // one job per wavefront of the first kFftWaveJobs
                const FftJob* g = a.fft_jobs[PASS - 1] + (size_t)wg * kFftWaveJobs;
                float* bufs = reinterpret_cast<float*>(lds4);
                float2 x[WaveGeom<FFTLOGN>::E];
                if (NW == kFftWaveJobs && g->flags == kFftGroupCols) {
                    fft_wave_load_cols<FFTLOGN>(g, bufs, x);
                    fft_wave_job<FFTLOGN, true, true>(a, g + wv,
                                                      bufs + wv * WaveGeom<FFTLOGN>::BUF, x);
                } else if (wv < kFftWaveJobs) {
                    fft_wave_job<FFTLOGN, PASS == 2 || WIDE>(
                        a, g + wv, bufs + wv * WaveGeom<FFTLOGN>::BUF, x);
                }
            } else {
                fft_job<FFTLOGN, 64 * NW, PASS == 2 || WIDE>(a, a.fft_jobs[PASS - 1] + wg,
                                                              reinterpret_cast<float2*>(lds4));
            }
            return;
        }
        wg -= nf;
    }
    const Tile tl = cst(PASS == 1 ? a.tiles1 : a.tiles2)[wg];
    const FrameDesc f = frame_of(a, tl.frame);
    // the tile's planes: tl.plane and the (tl.n_planes - 1) planes below it,
    // widest first, each over the same columns and band (one plane if 0)
    const int n_pl = GROUP && tl.n_planes > 1 ? tl.n_planes : 1;
    for (int pi = 0; pi < n_pl; ++pi) {
        if (pi > 0)
            __syncthreads();   // the previous plane's last LDS reads are done
        const int p = tl.plane - pi;
        const int r = cst(a.ladders)[f.ladder].r[p];
        const cptr_t w = (cptr_t)(a.weights + cst(a.ladders)[f.ladder].woff[p]);
        const float* src = PASS == 1 ? f.src : f.T + (long long)p * f.W * f.pitch;
        const int n = PASS == 1 ? f.H : f.W;                       // rows along the blur
        const int stride = PASS == 1 ? (int)f.src_stride : (int)f.pitch;
        const int ncols = PASS == 1 ? f.W : (int)f.pitch;
        const unsigned bytes = PASS == 1
                                   ? (unsigned)(((long long)(f.H - 1) * f.src_stride + f.W) * 4)
                                   : (unsigned)((long long)f.W * f.pitch * 4);
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(src, bytes);
        const int col0 = tl.cb * 64;
        (void)ncols;
        const int y0 = tl.band * (NW * S);
        const int base = y0 - r;
        const int nch = (2 * r + S) / S;   // tap chunks
        const int nload = nch + NW;        // row chunks X_0 .. X_{nch+NW-1}
        // the plane's taps go to LDS when they fit: each step then reads its S
        // weights as broadcast vector loads, with no scalar-load latency per step
        const bool w_lds = nch * S <= kLdsWeights;
        if (w_lds) {
            const float4* w4 = reinterpret_cast<const float4*>(a.weights + cst(a.ladders)[f.ladder].woff[p]);
            for (int q = tid; q < nch * S / 4; q += G::NT)
                wl4[q] = w4[q];
        }

        // X_0 .. X_NW into the ring, X_{NW+1} .. X_{NW+P} into registers.  Loads
        // past the last chunk fetch the last chunk again (never stored), so every
        // step issues the same loads.
#pragma unroll
        for (int j = 0; j <= NW; ++j) {
            float4 t[G::LPL];
            stage_load<S, NW, WIDE>(t, rs, tid, base, j, n, stride, col0);
            stage_store<S, NW>(lds4, j, t, tid);
        }
        float4 stg[P][G::LPL];
#pragma unroll
        for (int k = 0; k < P; ++k)
            stage_load<S, NW, WIDE>(stg[k], rs, tid, base, min(NW + 1 + k, nload - 1), n, stride, col0);
        __syncthreads();

        float acc[S], lo[S], hi[S], wr[S];
#pragma unroll
        for (int t = 0; t < S; ++t)
            acc[t] = 0.0f;
        lds_rows<S>(lo, lds, wv, lane);
        // step c: taps c*S .. c*S+S-1 on X_{w+c}, X_{w+c+1}; then publish
        // X_{NW+1+c} from staging register set c % P and refill that set
        auto step = [&](int c, float4 (&st)[G::LPL]) {
            // weights first: LDS returns in order, so the first products (with
            // `lo` and these weights) need not wait for the rows of `hi`
            if (w_lds) {
#pragma unroll
                for (int u = 0; u < S; u += 4) {
                    const float4 q = wl4[(c * S + u) / 4];
                    wr[u] = q.x;
                    wr[u + 1] = q.y;
                    wr[u + 2] = q.z;
                    wr[u + 3] = q.w;
                }
            } else {
#pragma unroll
                for (int u = 0; u < S; ++u)
                    wr[u] = to_vgpr(w[c * S + u]);
            }
            lds_rows<S>(hi, lds, (wv + c + 1) % G::Q, lane);
            fma_chunk_v<S>(acc, lo, hi, wr);
#pragma unroll
            for (int t = 0; t < S; ++t) {
                // the accumulators pass through an empty asm statement, so the
                // multiply-adds cannot sink past the barrier below (two steps'
                // operands live at once would cost occupancy)
                asm volatile("" : "+v"(acc[t]));
                lo[t] = hi[t];
            }
            const int j = NW + 1 + c;
            if (j < nload)
                stage_store<S, NW>(lds4, j % G::Q, st, tid);
            stage_load<S, NW, WIDE>(st, rs, tid, base, min(j + P, nload - 1), n, stride, col0);
            __syncthreads();
        };
        // whole groups of P steps issue the same loads every iteration, so each
        // wait covers exactly the oldest staged chunk
        int c = 0;
        for (; c + P <= nch; c += P) {
#pragma unroll
            for (int k = 0; k < P; ++k)
                step(c + k, stg[k]);
        }
#pragma unroll
        for (int k = 0; k < P - 1; ++k)
            if (c + k < nch)
                step(c + k, stg[k]);

        if (PASS == 1) {
            // T is stored transposed: output column x is a row of T.  The tile
            // (64 columns x NW*S outputs) goes through LDS (the ring is free after
            // the last barrier) so that consecutive threads write consecutive
            // 16-byte pieces of each T row; a direct store from the accumulators
            // would scatter every store instruction over 64 rows of T.
            constexpr int TS = NW * S + 4;   // LDS floats per column (padded)
            constexpr int Q4 = NW * S / 4;   // 16-byte pieces per column
            constexpr int NQ = 64 * Q4;
            static_assert(64 * TS <= G::Q * S * 64, "transpose tile fits the ring");
            float* tr = reinterpret_cast<float*>(lds4);
#pragma unroll
            for (int t = 0; t < S; t += 4)
                *reinterpret_cast<float4*>(tr + lane * TS + wv * S + t) =
                    make_float4(acc[t], acc[t + 1], acc[t + 2], acc[t + 3]);
            __syncthreads();
#pragma unroll
            for (int i = 0; i < (NQ + G::NT - 1) / G::NT; ++i) {
                const int q = tid + i * G::NT;
                if (NQ % G::NT == 0 || q < NQ) {
                    const int cx = q / Q4, y4 = q - cx * Q4;
                    const int x = col0 + cx, y = y0 + 4 * y4;
                    if (x < f.W && y < f.H) {
                        const float4 v = *reinterpret_cast<const float4*>(tr + cx * TS + 4 * y4);
                        float* __restrict__ dst = f.T + ((long long)p * f.W + x) * f.pitch + y;
                        if (y + 4 <= f.H) {
                            *reinterpret_cast<float4*>(dst) = v;
                        } else {
                            dst[0] = v.x;
                            if (y + 1 < f.H)
                                dst[1] = v.y;
                            if (y + 2 < f.H)
                                dst[2] = v.z;
                        }
                    }
                }
            }
        } else {
            // L rows are contiguous along the lanes: direct coalesced stores
            const int col = col0 + lane;
            const int o0 = y0 + wv * S;  // first output of this wave along the blur
            if (col < f.H) {
                float* __restrict__ dstp = f.L + (long long)p * f.W * f.pitch;
#pragma unroll
                for (int t = 0; t < S; ++t)
                    if (o0 + t < f.W)
                        dstp[(long long)(o0 + t) * f.pitch + col] = acc[t];
            }
        }
    }   // planes of the tile
}

// Lanes i-1 and i+1 of a wave.  Lanes 0 and 63 receive 0 from outside the
// wave; they are halo lanes whose results are never used.
__device__ __forceinline__ float lane_prev(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138,
                                                              0xf, 0xf, true));
}

__device__ __forceinline__ float lane_next(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130,
                                                              0xf, 0xf, true));
}

// Rows x0-1 .. x0+BN of column y of transposed plane p, loaded without
// branches: rows outside the frame are clamped (their values are replaced by
// -inf in dog_rows) and the row offset is forced into a scalar register.
template <int BN>
__device__ __forceinline__ void load_plane_rows(float (&v)[BN + 2], const FrameDesc& f, int p,
                                                int x0, unsigned voff, bool live = true)
{
    // !live: a buffer of 0 bytes, so the loads return 0 and touch no memory
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(f.L + (long long)p * f.W * f.pitch,
                                                 live ? (unsigned)((long long)f.W * f.pitch * 4) : 0u);
    const int stride4 = (int)(f.pitch * 4);
#pragma unroll
    for (int j = 0; j < BN + 2; ++j) {
        int x = x0 - 1 + j;
        x = x < 0 ? 0 : (x >= f.W ? f.W - 1 : x);
        v[j] = load_f32(rs, voff, __builtin_amdgcn_readfirstlane(x * stride4));
    }
}

// DoG of one scale over BN band rows plus a one-row halo on each side:
// D = sigma (La - Lb), -inf outside the frame; returns the 3x3 spatial maxima
// s3 and the centre values dc of the band rows.
template <int BN>
__device__ __forceinline__ void dog_rows(const float (&La)[BN + 2], const float (&Lb)[BN + 2],
                                         float sigma, int x0, int W, bool ycol, float (&s3)[BN],
                                         float (&dc)[BN])
{
    float hm[BN + 2];
#pragma unroll
    for (int j = 0; j < BN + 2; ++j) {
        const int x = x0 - 1 + j;
        const bool ok = ycol && x >= 0 && x < W;
        const float d = ok ? sigma * (La[j] - Lb[j]) : -INFINITY;
        hm[j] = fmaxf(d, fmaxf(lane_prev(d), lane_next(d)));
        if (j >= 1 && j <= BN)
            dc[j - 1] = d;
    }
#pragma unroll
    for (int j = 0; j < BN; ++j)
        s3[j] = fmaxf(hm[j], fmaxf(hm[j + 1], hm[j + 2]));
}

#define DOG_LDS_RECS 512

// Workgroup-local candidate buffer: survivors are appended in LDS and
// flushed with one global atomic per tile (a tile that overflows it is
// walked again, its records going straight to the global list).
struct CandSink {
    uint32_t* s_n;
    CandRec* s_rec;
    CandHeader* cand;
    CandRec* recs;
    uint32_t cap;
    CandRec* host_recs;   // pinned host copy of records [0, lim_h)
    uint32_t lim_h;       // min(cap, n_host)
};

// Append the voxels of one band row whose flag is set (wave ballot, prefix
// popcount, one atomic per wave).  LDS mode: to the workgroup's LDS buffer,
// counting (not storing) records beyond its capacity, so the walk issues no
// global memory operation besides its plane loads.  GLOBAL mode (a tile whose
// records overflowed the buffer, walked a second time): straight to the device
// list and, below lim_h, to the pinned host copy; *s_end keeps the largest end.
template <bool GLOBAL>
__device__ __forceinline__ void emit_rec(const CandSink& snk, uint32_t* s_end,
                                         const FrameDesc& f, int lane, int y, int x, int i,
                                         bool flag, float d)
{
    const unsigned long long bal = __ballot(flag);
    if (bal != 0ull) {
        const unsigned cnt = (unsigned)__popcll(bal);
        unsigned base = 0;
        if (lane == 0) {
            if (GLOBAL) {
                base = atomicAdd(&snk.cand->count, cnt);
                atomicMax(s_end, base + cnt);
            } else {
                base = atomicAdd(snk.s_n, cnt);
            }
        }
        base = __shfl(base, 0);
        if (flag) {
            CandRec rec;
            rec.frame = f.frame_id;
            rec.y = y;
            rec.x = x;
            rec.scale = i;
            rec.response = d;
            const unsigned idx = base + (unsigned)__popcll(bal & ((1ull << lane) - 1ull));
            if (GLOBAL) {
                if (idx < snk.cap)
                    snk.recs[idx] = rec;
                if (idx < snk.lim_h)
                    snk.host_recs[idx] = rec;
            } else if (idx < DOG_LDS_RECS) {
                snk.s_rec[idx] = rec;
            }
        }
    }
}

// Test the BN band rows of scale i: a voxel is kept iff it equals the maximum
// of its 3x3x3 neighbourhood and exceeds the threshold.  One ballot decides
// whether any row has a survivor; rows are then appended one by one.  The
// debug build also stores the DoG plane.
template <int BN, bool DBG, bool GLOBAL>
__device__ __forceinline__ void test_plane(const CandSink& snk, uint32_t* s_end,
                                           const FrameDesc& f, int lane, int y, int x0, int i,
                                           bool yout, const float (&dc)[BN],
                                           const float (&s3m)[BN], const float (&s3c)[BN],
                                           const float (&s3n)[BN], float thr, long long plane_sz)
{
    bool flag[BN];
    bool any = false;
#pragma unroll
    for (int j = 0; j < BN; ++j) {
        const int x = x0 + j;
        const bool inside = yout && x < f.W;
        const float m = fmaxf(s3m[j], fmaxf(s3c[j], s3n[j]));
        flag[j] = inside && dc[j] == m && dc[j] > thr;
        any = any || flag[j];
        if (DBG && inside)
            f.Ddbg[(long long)i * plane_sz + (long long)x * f.pitch + y] = dc[j];
    }
    if (__ballot(any) != 0ull) {
#pragma unroll
        for (int j = 0; j < BN; ++j)
            emit_rec<GLOBAL>(snk, s_end, f, lane, y, x0 + j, i, flag[j], dc[j]);
    }
}

// One wave's walk over all scales of its BN band rows (rows x0 .. x0+BN-1 of
// the transposed planes, lane = column y).  The band rows of the planes are
// held in a ring of NB buffers, plane p in buffer p mod NB: step i forms
// D_{i+1} from planes i+1 and i+2 while plane i+NB is loaded into the buffer
// that plane i left, so NB-2 planes are in flight ahead of the one the step
// waits for.  The loop is unrolled NB times so that every buffer index is a
// constant: the ring rotates by renaming, not by register moves (a move would
// wait for the load just issued).  Past the last plane the loads still issue,
// from a buffer of 0 bytes (they return 0 and fetch nothing), so every path
// issues the same loads and the waits count exactly.
template <int BN, int NB, bool DBG, bool GLOBAL>
__device__ __forceinline__ void nms_walk(const CandSink& snk, uint32_t* s_end,
                                         const FrameDesc& f, const DOG_CONSTANT_AS LadderDesc* ld,
                                         int lane, int y, bool ycol, bool yout, unsigned voff,
                                         int x0)
{
    const int k = ld->n_g - 1;
    const float thr = ld->thr;
    const long long plane_sz = (long long)f.W * f.pitch;
    float s3m[BN], s3c[BN], s3n[BN], dc[BN], dn[BN];
#pragma unroll
    for (int j = 0; j < BN; ++j)
        s3m[j] = -INFINITY;
    float L[NB][BN + 2];
#pragma unroll
    for (int p = 0; p < NB; ++p)
        load_plane_rows<BN>(L[p], f, p <= k ? p : k, x0, voff, p <= k);
    dog_rows<BN>(L[0], L[1], ld->sigma[0], x0, f.W, ycol, s3c, dc);
    for (int i0 = 0; i0 < k; i0 += NB) {
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const int i = i0 + m;
            if (i >= k)
                break;
            load_plane_rows<BN>(L[m], f, i + NB <= k ? i + NB : k, x0, voff, i + NB <= k);
            if (i + 1 < k) {
                dog_rows<BN>(L[(m + 1) % NB], L[(m + 2) % NB], ld->sigma[i + 1], x0, f.W, ycol,
                             s3n, dn);
            } else {
#pragma unroll
                for (int j = 0; j < BN; ++j) {
                    s3n[j] = -INFINITY;
                    dn[j] = -INFINITY;
                }
            }
            test_plane<BN, DBG, GLOBAL>(snk, s_end, f, lane, y, x0, i, yout, dc, s3m, s3c, s3n,
                                        thr, plane_sz);
#pragma unroll
            for (int j = 0; j < BN; ++j) {
                s3m[j] = s3c[j];
                s3c[j] = s3n[j];
                dc[j] = dn[j];
            }
        }
    }
}

// Plane buffers of the local-maximum walk: one plane in flight ahead of the
// step's two.  Measured on the 1024x1024 frame (9 planes, 4 rows per wave):
// 10.5 us with 3 buffers, 11.0 with 4, 12.2 with 5, 12.3 with 6.  With 3
// buffers and 4 waves per workgroup, 6 rows per wave took 9.9 us (100 VGPRs);
// 2, 4 and 8 rows 11.9, 10.5 and 12.6 us; 8 waves of 2 or 4 rows 11.6 and 11.8.
constexpr int kNmsRing = 3;

// Local maxima of the DoG cube with threshold, compacted into records.
// Tile = 62 output columns (y; lanes 1..62, lanes 0 and 63 are the halo)
// x (BN*NW) rows (x) of one frame; every wave walks all scales, appending its
// survivors to the workgroup's LDS buffer, which is then flushed with one
// global atomic.  A tile with more survivors than the buffer holds (plateaus
// of equal values) is walked again with every record going straight to the
// device list.  DBG also writes the DoG planes (parity tests only).
template <int BN, int NW, bool DBG, int NB>
__global__ void __launch_bounds__(64 * NW) k_nms(LaunchArgs a)
{
    static_assert(NB >= 3, "the ring holds two planes and the one in flight");
    __shared__ uint32_t s_n;
    __shared__ uint32_t s_base;
    __shared__ CandRec s_rec[DOG_LDS_RECS];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (threadIdx.x == 0) {
        s_n = 0u;
        s_base = 0u;
    }
    __syncthreads();
    const CandSink snk{&s_n, s_rec, a.cand, reinterpret_cast<CandRec*>(a.cand + 1), a.cap,
                       a.host_recs, a.cap < a.n_host ? a.cap : a.n_host};
    const Tile tl = my_tile(a.tiles3);
    const FrameDesc f = frame_of(a, tl.frame);
    const DOG_CONSTANT_AS LadderDesc* ld = cst(a.ladders) + f.ladder;
    const int y = tl.cb * DOG_NMS_COLS - 1 + lane;
    const bool ycol = y >= 0 && y < f.H;
    const bool yout = ycol && lane >= 1 && lane <= DOG_NMS_COLS;
    const unsigned voff = (unsigned)(ycol ? y : 0) * 4u;
    const int x0 = tl.band * (BN * NW) + wv * BN;
    if (x0 < f.W)  // wave-uniform
        nms_walk<BN, NB, DBG, false>(snk, &s_base, f, ld, lane, y, ycol, yout, voff, x0);
    __syncthreads();
    const uint32_t n = s_n;
    if (n <= DOG_LDS_RECS) {
        if (threadIdx.x == 0)
            s_base = n ? atomicAdd(&snk.cand->count, n) : 0u;
        __syncthreads();
        const uint32_t gbase = s_base;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t g = gbase + i;
            if (g < snk.cap)
                snk.recs[g] = s_rec[i];
            if (g < snk.lim_h)
                snk.host_recs[g] = s_rec[i];
        }
        if (threadIdx.x == 0)
            a.host_ends[blockIdx.x] = gbase + n;
    } else {
        // s_base (0 here) now keeps the largest end of the records written
        if (x0 < f.W)
            nms_walk<BN, NB, DBG, true>(snk, &s_base, f, ld, lane, y, ycol, yout, voff, x0);
        __syncthreads();
        if (threadIdx.x == 0)
            a.host_ends[blockIdx.x] = s_base;
    }
}

// dst[(p*H + y)*W + x] = src[(p*W + x)*pitch + y]: back to row-major planes.
__global__ void k_untranspose(const float* __restrict__ src, float* __restrict__ dst, int n_planes,
                              int H, int W, long long pitch)
{
    const long long total = (long long)n_planes * H * W;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long p = i / ((long long)H * W);
        const long long rem = i - p * H * W;
        const int yy = (int)(rem / W);
        const int xx = (int)(rem - (long long)yy * W);
        dst[i] = src[(p * W + xx) * pitch + yy];
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int n, uint32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

// ---------------------------------------------------------------- launchers

struct KernelSet {
    const void* pass1;
    const void* pass1w;   // pass 1 when every frame has 16-byte aligned rows and
                          // a width that is a multiple of 64 (nullptr: same as pass1)
    const void* pass2;
    const void* nms[2];     // [debug planes]
    int S, R, NW, BI, BN, NWN;
    int group;              // staged blur: a tile takes several planes (cost-balanced)
    // the blur passes with the transform-domain jobs of lines of 2^(7+i)
    // values in the same launch (nullptr: the job does not fit the ring)
    const void* pass1f[DOG_FFT_MERGED];
    const void* pass1wf[DOG_FFT_MERGED];
    const void* pass2f[DOG_FFT_MERGED];
};

// k_blur_lds with the transform jobs of lines of 2^LOGN values, if a job's
// LDS fits the ring of this geometry.
template <int PASS, int S, int NW, int P, bool WIDE, int LOGN>
static const void* merged_fn()
{
    if constexpr (fft_merged_lds<LOGN, NW>() <= (size_t)(NW + 2) * S * 256)
        return reinterpret_cast<const void*>(&k_blur_lds<PASS, S, NW, P, WIDE, LOGN>);
    else
        return nullptr;
}

template <int S, int NW, int P>
static void fill_merged(KernelSet& k)
{
    const void* f1[DOG_FFT_MERGED] = {merged_fn<1, S, NW, P, false, 7>(),
                                      merged_fn<1, S, NW, P, false, 8>(),
                                      merged_fn<1, S, NW, P, false, 9>(),
                                      merged_fn<1, S, NW, P, false, 10>()};
    const void* f1w[DOG_FFT_MERGED] = {merged_fn<1, S, NW, P, true, 7>(),
                                       merged_fn<1, S, NW, P, true, 8>(),
                                       merged_fn<1, S, NW, P, true, 9>(),
                                       merged_fn<1, S, NW, P, true, 10>()};
    const void* f2[DOG_FFT_MERGED] = {merged_fn<2, S, NW, P, true, 7>(),
                                      merged_fn<2, S, NW, P, true, 8>(),
                                      merged_fn<2, S, NW, P, true, 9>(),
                                      merged_fn<2, S, NW, P, true, 10>()};
    for (int i = 0; i < DOG_FFT_MERGED; ++i) {
        k.pass1f[i] = f1[i];
        k.pass1wf[i] = f1w[i];
        k.pass2f[i] = f2[i];
    }
}

template <int S, int NW, int P, int BN, int NWN, int GROUP = 0>
static KernelSet make_lds_set()
{
    KernelSet k;
    k.group = GROUP;
    if (GROUP) {
        for (int i = 0; i < DOG_FFT_MERGED; ++i)
            k.pass1f[i] = k.pass1wf[i] = k.pass2f[i] = nullptr;
    } else {
        fill_merged<S, NW, P>(k);
    }
    k.pass1 = reinterpret_cast<const void*>(&k_blur_lds<1, S, NW, P, false, 0, GROUP != 0>);
    k.pass1w = reinterpret_cast<const void*>(&k_blur_lds<1, S, NW, P, true, 0, GROUP != 0>);
    k.pass2 = reinterpret_cast<const void*>(&k_blur_lds<2, S, NW, P, true, 0, GROUP != 0>);
    k.nms[0] = reinterpret_cast<const void*>(&k_nms<BN, NWN, false, kNmsRing>);
    k.nms[1] = reinterpret_cast<const void*>(&k_nms<BN, NWN, true, kNmsRing>);
    k.S = S;
    k.R = P;
    k.NW = NW;
    k.BI = 1;
    k.BN = BN;
    k.NWN = NWN;
    return k;
}

template <int S, int R, int NW, int BI, int BN, int NWN>
static KernelSet make_set()
{
    KernelSet k;
    k.group = 0;
    for (int i = 0; i < DOG_FFT_MERGED; ++i)
        k.pass1f[i] = k.pass1wf[i] = k.pass2f[i] = nullptr;
    k.pass1w = nullptr;
    k.pass1 = reinterpret_cast<const void*>(&k_pass1<S, R, NW, BI>);
    k.pass2 = reinterpret_cast<const void*>(&k_pass2<S, R, NW, BI>);
    k.nms[0] = reinterpret_cast<const void*>(&k_nms<BN, NWN, false, kNmsRing>);
    k.nms[1] = reinterpret_cast<const void*>(&k_nms<BN, NWN, true, kNmsRing>);
    k.S = S;
    k.R = R;
    k.NW = NW;
    k.BI = BI;
    k.BN = BN;
    k.NWN = NWN;
    return k;
}

// Variants available to the autotuner: (S outputs per lane, R ring buffers,
// waves per workgroup, strips per wave) for the blur passes and (rows per
// wave, waves) for the local-maximum kernel.  The last three run the staged
// kernels of variants 8, 9 and 13 with cost-balanced tiles: each tile takes
// a run of consecutive planes whose tap chunks add up to about those of the
// widest plane (the kernels are the same; only the host's tile tables
// differ), so every workgroup runs a long chain of steps.
static const KernelSet kSets[] = {
    make_set<12, 4, 4, 1, 4, 4>(),
    make_set<12, 6, 4, 1, 4, 4>(),
    make_set<16, 3, 4, 1, 4, 4>(),
    make_set<16, 4, 4, 1, 4, 4>(),
    make_set<16, 6, 4, 1, 4, 4>(),
    make_set<20, 3, 4, 1, 4, 4>(),
    make_set<12, 8, 4, 1, 4, 4>(),
    make_set<24, 3, 4, 1, 8, 4>(),
    make_lds_set<16, 4, 2, 6, 4>(),
    make_lds_set<16, 4, 4, 6, 4>(),
    make_lds_set<12, 4, 2, 6, 4>(),
    make_lds_set<8, 8, 2, 6, 4>(),
    make_lds_set<16, 8, 2, 6, 4>(),
    make_lds_set<16, 2, 2, 6, 4>(),
    make_lds_set<16, 4, 2, 6, 4, 1>(),
    make_lds_set<16, 4, 4, 6, 4, 1>(),
    make_lds_set<16, 2, 2, 6, 4, 1>(),
};

}  // namespace dog

extern "C" {

int dogk_num_variants() { return (int)(sizeof(dog::kSets) / sizeof(dog::kSets[0])); }

void dogk_variant_geometry(int v, int* S, int* NW, int* BI, int* BN, int* NWN)
{
    const dog::KernelSet& k = dog::kSets[v];
    *S = k.S;
    *NW = k.NW;
    *BI = k.BI;
    *BN = k.BN;
    *NWN = k.NWN;
}

int dogk_variant_ring(int v) { return dog::kSets[v].R; }

int dogk_variant_group(int v) { return dog::kSets[v].group; }

// Launch blur pass `pass` (1 or 2) on `stream`, one workgroup per tile of
// its table, after args->n_fft[pass - 1] workgroups of transform-domain jobs
// of lines of 2^fft_logn values when fft_logn > 0 (the launch must then have
// such jobs and the variant a merged kernel for them); a pass with no
// workgroups is not launched.  Pass 1 also clears the candidate count, so
// without pass-1 workgroups a fill kernel does.  wide1: every frame's rows
// are 16-byte aligned and its width is a multiple of 64, so pass 1 may use
// 16-byte loads.  If ev is non-NULL, ev[0] and ev[1] take the start and end
// of the pass's execution (the dispatch's own timestamps, so the launch gap
// before a kernel is not counted).
hipError_t dogk_launch_pass(int variant, const dog::LaunchArgs* args, int pass, int grid,
                            int fft_logn, int wide1, hipStream_t stream, hipEvent_t* ev)
{
    const dog::KernelSet& k = dog::kSets[variant];
    const void* fn = pass == 1 ? (wide1 && k.pass1w ? k.pass1w : k.pass1) : k.pass2;
    if (fft_logn > 0) {
        const int i = fft_logn - 7;
        if (i < 0 || i >= DOG_FFT_MERGED)
            return hipErrorInvalidValue;
        fn = pass == 1 ? (wide1 ? k.pass1wf[i] : k.pass1f[i]) : k.pass2f[i];
        if (!fn)
            return hipErrorInvalidValue;
        grid += args->n_fft[pass - 1];
    }
    void* params[] = {const_cast<dog::LaunchArgs*>(args)};
    if (pass == 1 && grid <= 0) {
        hipLaunchKernelGGL(dog::k_fill_u32, dim3(1), dim3(64), 0, stream, &args->cand->count, 1, 0u);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (grid <= 0)
        return hipSuccess;
    return ev ? hipExtLaunchKernel(fn, dim3(grid), dim3(64 * k.NW), params, 0, stream, ev[0],
                                   ev[1], 0)
              : hipLaunchKernel(fn, dim3(grid), dim3(64 * k.NW), params, 0, stream);
}

// Whether variant v's blur passes can run transform-domain jobs of lines of
// 2^logn values in their own launches.
int dogk_variant_merges_fft(int v, int logn)
{
    const int i = logn - 7;
    if (i < 0 || i >= DOG_FFT_MERGED)
        return 0;
    const dog::KernelSet& k = dog::kSets[v];
    return k.pass1f[i] && k.pass1wf[i] && k.pass2f[i] ? 1 : 0;
}

// The local-maximum kernel (timed by ev[0], ev[1] when ev is non-NULL).
hipError_t dogk_launch_nms_ev(int variant, const dog::LaunchArgs* args, int grid3, int debug,
                              hipStream_t stream, hipEvent_t* ev)
{
    const dog::KernelSet& k = dog::kSets[variant];
    void* params[] = {const_cast<dog::LaunchArgs*>(args)};
    const void* fn = k.nms[debug ? 1 : 0];
    return ev ? hipExtLaunchKernel(fn, dim3(grid3), dim3(64 * k.NWN), params, 0, stream, ev[0],
                                   ev[1], 0)
              : hipLaunchKernel(fn, dim3(grid3), dim3(64 * k.NWN), params, 0, stream);
}

hipError_t dogk_launch_nms(int variant, const dog::LaunchArgs* args, int grid3, int max_gauss,
                           int debug, hipStream_t stream)
{
    const dog::KernelSet& k = dog::kSets[variant];
    void* params[] = {const_cast<dog::LaunchArgs*>(args)};
    (void)max_gauss;
    return hipLaunchKernel(k.nms[debug ? 1 : 0], dim3(grid3),
                           dim3(64 * k.NWN), params, 0, stream);
}

// Resident workgroups per CU of each kernel of a variant.
hipError_t dogk_occupancy(int variant, int* wg1, int* wg2, int* wg3)
{
    const dog::KernelSet& k = dog::kSets[variant];
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(wg1, k.pass1, 64 * k.NW, 0);
    if (e != hipSuccess)
        return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(wg2, k.pass2, 64 * k.NW, 0);
    if (e != hipSuccess)
        return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(wg3, k.nms[0], 64 * k.NWN, 0);
}

hipError_t dogk_untranspose(const float* src, float* dst, int n_planes, int H, int W,
                            long long pitch, hipStream_t stream)
{
    const long long total = (long long)n_planes * H * W;
    long long blocks = (total + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(dog::k_untranspose, dim3((unsigned)blocks), dim3(256), 0, stream, src, dst,
                       n_planes, H, W, pitch);
    return hipGetLastError();
}

hipError_t dogk_fill_u32(uint32_t* p, int n, uint32_t v, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(dog::k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

}  // extern "C"
