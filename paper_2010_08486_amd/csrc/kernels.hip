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
// value feeds S fused multiply-adds.  Reflection at the borders only ever
// applies to the walking direction, where the row index is uniform, so the
// interior path has no per-lane boundary logic at all.
//
// All three kernels are persistent: a fixed grid of workgroups pulls tiles
// from an atomic counter, so one captured launch sequence serves batches of
// any composition.  Each kernel clears the counter of the kernel two steps
// ahead in the sequence (pass 1 clears the nms counter and the candidate
// count, pass 2 clears pass 1's, nms clears pass 2's); a kernel never touches
// its own counter while it runs.
#include <hip/hip_runtime.h>

#include "dog_internal.h"

// Pointers into the constant (scalar-load) address space.  The qualifier only
// exists for the device compilation pass; the host pass of this file sees
// plain pointers.
#if defined(__HIP_DEVICE_COMPILE__)
#define DOG_CONSTANT_AS __attribute__((address_space(4)))
#else
#define DOG_CONSTANT_AS
#endif

namespace dog {

// Half-sample symmetric reflection into [0, n), period 2n.
__device__ __forceinline__ int refl(int t, int n)
{
    if ((unsigned)t < (unsigned)n)
        return t;
    const int p = 2 * n;
    int u = t % p;
    if (u < 0)
        u += p;
    return u < n ? u : p - 1 - u;
}

// Scalar view of the launch tables: they are read-only during a launch and
// indexed uniformly, so their fields land in scalar registers.
template <class T>
__device__ __forceinline__ const DOG_CONSTANT_AS T* cst(const T* p)
{
    return (const DOG_CONSTANT_AS T*)p;
}

// Last unit whose first_tile <= tile (units sorted by first_tile).
__device__ __forceinline__ int find_unit(const WorkUnit* units, int n, int tile)
{
    const DOG_CONSTANT_AS WorkUnit* u = cst(units);
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (u[mid].first_tile <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Scalar (SMEM) view of the wave-uniform weight vectors.
typedef const DOG_CONSTANT_AS float* cptr_t;


// Buffer resource over one plane: raw (unswizzled) dword loads with a scalar
// row offset and a per-lane column offset; the hardware range check returns 0
// for any byte offset at or beyond `bytes` instead of touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

// v[m] = column c of row (row0 + m), m = 0..S-1.  Interior rows: vo[m] =
// 4c + m*stride4 (per-lane, loop-invariant) plus one scalar offset per chunk.
// Border rows: each row is reflected into [0, n) and addressed through the
// scalar offset, with vo[0] = 4c.  stride4 = row pitch in bytes.
template <int S, bool INTERIOR>
__device__ __forceinline__ void load_rows(float (&v)[S], __amdgpu_buffer_rsrc_t rs, int stride4,
                                          const unsigned (&vo)[S], int row0, int n)
{
#pragma unroll
    for (int m = 0; m < S; ++m) {
        unsigned bits;
        if (INTERIOR)
            bits = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)vo[m], row0 * stride4, 0);
        else
            bits = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)vo[0], refl(row0 + m, n) * stride4,
                                                        0);
        v[m] = __builtin_bit_cast(float, bits);
    }
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

// nch chunks of S taps over rows base .. base + (nch+1)*S - 1; three row
// buffers rotate so the loads of chunk ch+2 are in flight while chunk ch is
// multiplied.  Reads rows up to base + (nch+2)*S - 1.
template <int S, bool INTERIOR>
__device__ __forceinline__ void blur_chunks(__amdgpu_buffer_rsrc_t rs, int stride4, int n,
                                            unsigned c, int base, int nch, cptr_t w,
                                            float (&acc)[S])
{
    unsigned voff[S];
#pragma unroll
    for (int m = 0; m < S; ++m)
        voff[m] = 4u * c + (INTERIOR ? (unsigned)(m * stride4) : 0u);
    float A[S], B[S], C[S];
    load_rows<S, INTERIOR>(A, rs, stride4, voff, base, n);
    load_rows<S, INTERIOR>(B, rs, stride4, voff, base + S, n);
    int ch = 0;
    for (; ch + 3 <= nch; ch += 3) {
        load_rows<S, INTERIOR>(C, rs, stride4, voff, base + (ch + 2) * S, n);
        fma_chunk<S>(acc, A, B, w + ch * S);
        load_rows<S, INTERIOR>(A, rs, stride4, voff, base + (ch + 3) * S, n);
        fma_chunk<S>(acc, B, C, w + (ch + 1) * S);
        load_rows<S, INTERIOR>(B, rs, stride4, voff, base + (ch + 4) * S, n);
        fma_chunk<S>(acc, C, A, w + (ch + 2) * S);
    }
    const int rem = nch - ch;
    if (rem == 2)
        load_rows<S, INTERIOR>(C, rs, stride4, voff, base + (ch + 2) * S, n);
    if (rem >= 1)
        fma_chunk<S>(acc, A, B, w + ch * S);
    if (rem == 2)
        fma_chunk<S>(acc, B, C, w + (ch + 1) * S);
}

// acc[t] = sum_{j=0}^{2r} w[j] * col[refl(y0 - r + t + j)], t = 0..S-1, where
// col[m] is column c of row m of the plane behind `rs`.  Taps are accumulated in ascending order, so
// every output sees the same summation order whatever the tile shape; w must
// be zero-padded up to ceil((2r+1)/S)*S.
template <int S>
__device__ __forceinline__ void blur_strip(__amdgpu_buffer_rsrc_t rs, int stride4, int n, int c,
                                           int y0, int r, const float* w, float (&acc)[S])
{
    const int base = y0 - r;
    const int nch = (2 * r + S) / S;
#pragma unroll
    for (int t = 0; t < S; ++t)
        acc[t] = 0.0f;
    const cptr_t cw = (cptr_t)w;
    if (base >= 0 && base + (nch + 2) * S <= n)
        blur_chunks<S, true>(rs, stride4, n, (unsigned)c, base, nch, cw, acc);
    else
        blur_chunks<S, false>(rs, stride4, n, (unsigned)c, base, nch, cw, acc);
}

// Pull the next tile id for the whole workgroup.
__device__ __forceinline__ int next_tile(uint32_t* ctr, int* s_tile)
{
    if (threadIdx.x == 0)
        *s_tile = (int)atomicAdd(ctr, 1u);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(*s_tile);
    __syncthreads();
    return t;
}

// Pass 1: T_p = column blur of the input frame, stored transposed.
// Tile = 64 columns x (S*NW*BI) rows of one (frame, plane) unit.
template <int S, int NW, int BI>
__global__ void __launch_bounds__(64 * NW) k_pass1(LaunchArgs a)
{
    __shared__ int s_tile;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    constexpr int BAND = S * NW * BI;
    for (;;) {
        const int tile = next_tile(&a.counters->pass1, &s_tile);
        if (tile >= a.total1)
            break;
        if (tile == 0 && threadIdx.x == 0) {
            a.counters->nms = 0u;
            a.cand->count = 0u;
        }
        const WorkUnit u = cst(a.units1)[find_unit(a.units1, a.n_units1, tile)];
        const int lt = tile - u.first_tile;
        const int cb = lt / u.n_band;
        const int band = lt - cb * u.n_band;
        const FrameDesc f = cst(a.frames)[u.frame];
        const int p = u.plane;
        const int r = cst(a.ladders)[f.ladder].r[p];
        const float* w = a.weights + cst(a.ladders)[f.ladder].woff[p];
        const int col = cb * 64 + lane;
        const __amdgpu_buffer_rsrc_t rs =
            plane_rsrc(f.src, (unsigned)(((long long)(f.H - 1) * f.src_stride + f.W) * 4));
        const int stride4 = (int)(f.src_stride * 4);
        if (col < f.W) {
            for (int q = 0; q < BI; ++q) {
                const int y0 = band * BAND + (q * NW + wv) * S;
                if (y0 >= f.H)
                    break;
                float acc[S];
                blur_strip<S>(rs, stride4, f.H, col, y0, r, w, acc);
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
template <int S, int NW, int BI>
__global__ void __launch_bounds__(64 * NW) k_pass2(LaunchArgs a)
{
    __shared__ int s_tile;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    constexpr int BAND = S * NW * BI;
    for (;;) {
        const int tile = next_tile(&a.counters->pass2, &s_tile);
        if (tile >= a.total2)
            break;
        if (tile == 0 && threadIdx.x == 0)
            a.counters->pass1 = 0u;
        const WorkUnit u = cst(a.units2)[find_unit(a.units2, a.n_units2, tile)];
        const int lt = tile - u.first_tile;
        const int cb = lt / u.n_band;
        const int band = lt - cb * u.n_band;
        const FrameDesc f = cst(a.frames)[u.frame];
        const int p = u.plane;
        const int r = cst(a.ladders)[f.ladder].r[p];
        const float* w = a.weights + cst(a.ladders)[f.ladder].woff[p];
        const __amdgpu_buffer_rsrc_t rs = plane_rsrc(f.T + (long long)p * f.W * f.pitch,
                                                     (unsigned)((long long)f.W * f.pitch * 4));
        const int stride4 = (int)(f.pitch * 4);
        float* __restrict__ dstp = f.L + (long long)p * f.W * f.pitch;
        const int col = cb * 64 + lane;
        if (col < f.H) {
            for (int q = 0; q < BI; ++q) {
                const int x0 = band * BAND + (q * NW + wv) * S;
                if (x0 >= f.W)
                    break;
                float acc[S];
                blur_strip<S>(rs, stride4, f.W, col, x0, r, w, acc);
#pragma unroll
                for (int t = 0; t < S; ++t)
                    if (x0 + t < f.W)
                        dstp[(long long)(x0 + t) * f.pitch + col] = acc[t];
            }
        }
    }
}

// DoG of one scale over a band of BN rows plus a one-row halo on each side:
// loads L_{i+1} (rows x0-1 .. x0+BN), forms D_i = sigma_i (L_i - L_{i+1}) with
// -inf outside the frame, and returns the 3x3 spatial maxima s3 and the
// centre values dc of the BN band rows.  Lp holds L_i on entry, L_{i+1} on exit.
template <int BN>
__device__ __forceinline__ void dog_plane(const float* __restrict__ Lnext, long long pitch, int W,
                                          int x0, int y, bool ycol, float sigma,
                                          float (&Lp)[BN + 2], float (&s3)[BN], float (&dc)[BN])
{
    float hm[BN + 2];
#pragma unroll
    for (int j = 0; j < BN + 2; ++j) {
        const int x = x0 - 1 + j;
        const bool ok = ycol && x >= 0 && x < W;
        const float ln = ok ? Lnext[(long long)x * pitch + y] : 0.0f;
        const float d = ok ? sigma * (Lp[j] - ln) : -INFINITY;
        Lp[j] = ln;
        const float up = __shfl_up(d, 1);
        const float dn = __shfl_down(d, 1);
        hm[j] = fmaxf(d, fmaxf(up, dn));
        if (j >= 1 && j <= BN)
            dc[j - 1] = d;
    }
#pragma unroll
    for (int j = 0; j < BN; ++j)
        s3[j] = fmaxf(hm[j], fmaxf(hm[j + 1], hm[j + 2]));
}

// Local maxima of the DoG cube with threshold, compacted into records.
// Tile = 62 output columns (y; lanes 1..62, lanes 0 and 63 are the halo)
// x (BN*NW) rows (x) of one frame; every wave walks all scales.
template <int BN, int NW>
__global__ void __launch_bounds__(64 * NW) k_nms(LaunchArgs a)
{
    __shared__ int s_tile;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    CandRec* __restrict__ recs = reinterpret_cast<CandRec*>(a.cand + 1);
    for (;;) {
        const int tile = next_tile(&a.counters->nms, &s_tile);
        if (tile >= a.total3)
            break;
        if (tile == 0 && threadIdx.x == 0)
            a.counters->pass2 = 0u;
        const WorkUnit u = cst(a.units3)[find_unit(a.units3, a.n_units3, tile)];
        const int lt = tile - u.first_tile;
        const int cb = lt / u.n_band;
        const int band = lt - cb * u.n_band;
        const FrameDesc f = cst(a.frames)[u.frame];
        const DOG_CONSTANT_AS LadderDesc* ld = cst(a.ladders) + f.ladder;
        const int k = ld->n_g - 1;
        const float thr = ld->thr;
        const int y = cb * DOG_NMS_COLS - 1 + lane;
        const bool ycol = y >= 0 && y < f.H;
        const bool yout = ycol && lane >= 1 && lane <= DOG_NMS_COLS;
        const int x0 = band * (BN * NW) + wv * BN;
        if (x0 < f.W) {  // wave-uniform
            const long long plane_sz = (long long)f.W * f.pitch;
            float Lp[BN + 2];
#pragma unroll
            for (int j = 0; j < BN + 2; ++j) {
                const int x = x0 - 1 + j;
                Lp[j] = (ycol && x >= 0 && x < f.W) ? f.L[(long long)x * f.pitch + y] : 0.0f;
            }
            float s3m[BN], s3c[BN], s3n[BN], dc[BN], dn[BN];
#pragma unroll
            for (int j = 0; j < BN; ++j)
                s3m[j] = -INFINITY;
            dog_plane<BN>(f.L + plane_sz, f.pitch, f.W, x0, y, ycol, ld->sigma[0], Lp, s3c, dc);
            for (int i = 0; i < k; ++i) {
                if (i + 1 < k) {
                    dog_plane<BN>(f.L + (long long)(i + 2) * plane_sz, f.pitch, f.W, x0, y, ycol,
                                  ld->sigma[i + 1], Lp, s3n, dn);
                } else {
#pragma unroll
                    for (int j = 0; j < BN; ++j) {
                        s3n[j] = -INFINITY;
                        dn[j] = -INFINITY;
                    }
                }
#pragma unroll
                for (int j = 0; j < BN; ++j) {
                    const int x = x0 + j;
                    const float m = fmaxf(s3m[j], fmaxf(s3c[j], s3n[j]));
                    const bool flag = yout && x < f.W && dc[j] == m && dc[j] > thr;
                    if (f.Ddbg != nullptr && yout && x < f.W)
                        f.Ddbg[(long long)i * plane_sz + (long long)x * f.pitch + y] = dc[j];
                    const unsigned long long bal = __ballot(flag);
                    if (bal != 0ull) {
                        unsigned base = 0;
                        if (lane == 0)
                            base = atomicAdd(&a.cand->count, (unsigned)__popcll(bal));
                        base = __shfl(base, 0);
                        if (flag) {
                            const unsigned idx =
                                base + (unsigned)__popcll(bal & ((1ull << lane) - 1ull));
                            if (idx < a.cap) {
                                CandRec rec;
                                rec.frame = f.frame_id;
                                rec.y = y;
                                rec.x = x;
                                rec.scale = i;
                                rec.response = dc[j];
                                recs[idx] = rec;
                            }
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < BN; ++j) {
                    s3m[j] = s3c[j];
                    s3c[j] = s3n[j];
                    dc[j] = dn[j];
                }
            }
        }
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
    const void* pass2;
    const void* nms;
    int S, NW, BI, BN, NWN;
};

template <int S, int NW, int BI, int BN, int NWN>
static KernelSet make_set()
{
    KernelSet k;
    k.pass1 = reinterpret_cast<const void*>(&k_pass1<S, NW, BI>);
    k.pass2 = reinterpret_cast<const void*>(&k_pass2<S, NW, BI>);
    k.nms = reinterpret_cast<const void*>(&k_nms<BN, NWN>);
    k.S = S;
    k.NW = NW;
    k.BI = BI;
    k.BN = BN;
    k.NWN = NWN;
    return k;
}

// Variants available to the autotuner: (S, waves, strips per wave) for the
// blur passes and (rows, waves) for the local-maximum kernel.
static const KernelSet kSets[] = {
    make_set<8, 4, 2, 16, 4>(),
    make_set<8, 4, 4, 16, 4>(),
    make_set<8, 4, 8, 16, 4>(),
    make_set<8, 4, 1, 16, 4>(),
    make_set<4, 4, 4, 16, 4>(),
    make_set<12, 4, 2, 16, 4>(),
    make_set<16, 4, 1, 16, 4>(),
    make_set<8, 4, 16, 16, 4>(),
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

// Launch pass 1, pass 2 and the local-maximum kernel on `stream` with the
// given persistent grid sizes.  Returns the first launch error.
hipError_t dogk_launch_sequence(int variant, const dog::LaunchArgs* args, int grid1, int grid2,
                                int grid3, hipStream_t stream)
{
    const dog::KernelSet& k = dog::kSets[variant];
    void* params[] = {const_cast<dog::LaunchArgs*>(args)};
    hipError_t e = hipLaunchKernel(k.pass1, dim3(grid1), dim3(64 * k.NW), params, 0, stream);
    if (e != hipSuccess)
        return e;
    e = hipLaunchKernel(k.pass2, dim3(grid2), dim3(64 * k.NW), params, 0, stream);
    if (e != hipSuccess)
        return e;
    return hipLaunchKernel(k.nms, dim3(grid3), dim3(64 * k.NWN), params, 0, stream);
}

hipError_t dogk_launch_nms(int variant, const dog::LaunchArgs* args, int grid3, hipStream_t stream)
{
    const dog::KernelSet& k = dog::kSets[variant];
    void* params[] = {const_cast<dog::LaunchArgs*>(args)};
    return hipLaunchKernel(k.nms, dim3(grid3), dim3(64 * k.NWN), params, 0, stream);
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
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(wg3, k.nms, 64 * k.NWN, 0);
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
