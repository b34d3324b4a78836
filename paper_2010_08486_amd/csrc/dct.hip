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
// A job blurs two lines that are consecutive rows or columns of its input
// (one complex sequence) and produces, from one forward transform, the lines
// of every plane it lists.  Lines of 512, 1024 and 2048 values run one job
// per wavefront, the FFT in registers with two exchanges through the wave's own
// LDS (fft_wave.h); other lengths one job per workgroup, the FFT in the
// workgroup's LDS (fft_job.h).  The separable passes of a transform-domain
// plane run along x first, so that every job writes whole rows:
//   pass 1: the rows of the frame X[y][x] (lines along x), one forward
//           transform, then every transform-domain plane p, each output line
//           a row of U_p[y][x] (kept in the slot of the plane's T_p);
//   pass 2: per plane, the columns of U_p (lines along y), output lines rows
//           of L_p[x][y], the layout of the direct pass 2.
// The jobs of a pass run either in a launch of their own (this file) or in
// the launch of the direct blur pass, before its tiles (kernels.hip).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "dct.h"
#include "fft_job.h"
#include "fft_wave.h"

namespace dog {

namespace {
constexpr int kNT = 256;   // threads per job
}  // namespace

// One workgroup per job, or per kFftWaveJobs wave jobs.
template <int LOGN, bool VEC>
__global__ void __launch_bounds__(kNT) k_fft_blur(LaunchArgs a, const FftJob* __restrict__ jobs)
{
    extern __shared__ __align__(16) float2 lds[];
    if constexpr (fft_wave_len(LOGN)) {
        static_assert(kNT == 64 * kFftWaveJobs, "one job per wavefront");
        const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const FftJob* g = jobs + (size_t)blockIdx.x * kFftWaveJobs;
        float* bufs = reinterpret_cast<float*>(lds);
        float2 x[WaveGeom<LOGN>::E];
        if (g->flags == kFftGroupCols) {
            fft_wave_load_cols<LOGN>(g, bufs, x);
            fft_wave_job<LOGN, VEC, true>(a, g + w, bufs + w * WaveGeom<LOGN>::BUF, x);
        } else {
            fft_wave_job<LOGN, VEC>(a, g + w, bufs + w * WaveGeom<LOGN>::BUF, x);
        }
    } else {
        fft_job<LOGN, kNT, VEC>(a, jobs + blockIdx.x, lds);
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
    if (N == 512)
        return dog::WaveGeom<9>::LDS_BYTES;
    if (N == 1024)
        return dog::WaveGeom<10>::LDS_BYTES;
    if (N == 2048)
        return dog::WaveGeom<11>::LDS_BYTES;
    return ((size_t)N + (size_t)N / 16 + (size_t)N / 2 + (size_t)N) * sizeof(float2);
}

hipError_t dogk_fft_blur(const dog::LaunchArgs* args, const dog::FftJob* d_jobs, int n_jobs,
                         int logn, int vec, hipStream_t stream, hipEvent_t* ev)
{
    if (n_jobs <= 0)
        return hipSuccess;
    if (logn < 6 || logn > 11 || n_jobs % dog::fft_jobs_per_group(logn) != 0)
        return hipErrorInvalidValue;
    const int grid = n_jobs / dog::fft_jobs_per_group(logn);
    const void* const table[6] = {dog::fft_fn<6>(vec),  dog::fft_fn<7>(vec),
                                  dog::fft_fn<8>(vec),  dog::fft_fn<9>(vec),
                                  dog::fft_fn<10>(vec), dog::fft_fn<11>(vec)};
    const void* fn = table[logn - 6];
    const size_t lds_bytes = dogk_fft_lds_bytes(1 << logn);
    // dynamic LDS each instance has been allowed
    static size_t allowed[6][2] = {};
    size_t& ok = allowed[logn - 6][vec ? 1 : 0];
    if (lds_bytes > ok) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds_bytes);
        if (e != hipSuccess)
            return e;
        ok = lds_bytes;
    }
    const dog::FftJob* jobs = d_jobs;
    void* params[] = {const_cast<dog::LaunchArgs*>(args), &jobs};
    return ev ? hipExtLaunchKernel(fn, dim3(grid), dim3(256), params, lds_bytes, stream, ev[0],
                                   ev[1], 0)
              : hipLaunchKernel(fn, dim3(grid), dim3(256), params, lds_bytes, stream);
}

}  // extern "C"
