// Transform-domain blur (dct.hip): one workgroup's job.  Not part of the
// public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dog_internal.h"

namespace dog {

constexpr int kFftLines = 2;        // lines per job (one complex sequence)
constexpr int kFftMaxN = 2048;      // longest line
constexpr int kFftMaxPlanes = 16;   // planes one job produces from one forward transform
constexpr int kFftWaveJobs = 4;     // wave jobs per workgroup (one per wavefront, one plane each)

// FftJob::flags of the first of kFftWaveJobs wave jobs that are four column
// jobs of one input with line pairs line0, + 2, + 4, + 6 from a multiple of 8
// (16-byte aligned row pieces): one workgroup loads their lines together.
constexpr int kFftGroupCols = 1;

// Line lengths (log2) whose jobs run one per wavefront (fft_wave.h); the
// others run one per workgroup of 256 threads (fft_job.h).
constexpr bool fft_wave_len(int logn) { return logn >= 9 && logn <= 11; }
// Jobs per workgroup of the transform launches for lines of 2^logn values.
constexpr int fft_jobs_per_group(int logn) { return fft_wave_len(logn) ? kFftWaveJobs : 1; }
// float2 entries of the per-lane factor tables a wave job reads after the
// post-twiddles: log2 E + log2 A rows of 64, N = 64 E, A = 16 (E >= 16) or 8.
constexpr int fft_wave_table(int logn)
{
    return fft_wave_len(logn) ? ((logn - 6) + (logn >= 10 ? 4 : 3)) * 64 : 0;
}

// Outputs and transfer functions of the planes a group of jobs produces.
struct FftPlaneSet {
    float* out[kFftMaxPlanes];
    const float* h[kFftMaxPlanes];   // per plane: transfer function H[k] / N, k = 0..N-1
};

// Blur of kFftLines consecutive lines of length N (a power of two) by the
// kernels of n_planes planes (none: a padding job that does nothing).  The
// lines are rows line0 + l of the input (in_rows: element n of line l is
// in[(line0 + l) * in_pitch + n]) or its columns (element n of line l is
// in[n * in_pitch + line0 + l]).  Output line l of plane q is the row
// planes->out[q] + (line0 + l) * out_pitch.
struct FftJob {
    const float* in;         // NULL: the pixels of frame `frame` of the launch
    const float2* tw;        // N/2 twiddles exp(-2 pi i t / N)
    const float2* post;      // N twiddles exp(-i pi k / (2N)), then fft_wave_table(log2 N) more
    int32_t in_pitch;
    int32_t N;
    int32_t in_rows;
    int32_t line0;
    int32_t frame;
    int32_t n_planes;
    int32_t flags;           // first job of a group: kFftGroupCols or 0
    int32_t out_pitch;
    const FftPlaneSet* planes;   // the n_planes planes' outputs and transfer functions
};

}  // namespace dog

extern "C" {
size_t dogk_fft_lds_bytes(int N);
// n_jobs jobs whose lines all have 2^logn values (6 <= logn <= 11), a
// multiple of fft_jobs_per_group(logn) (padding jobs have no planes).  vec:
// every job's input rows hold its lines at 8-byte aligned addresses (pitch
// and line0 even, base 8-byte aligned); else 4-byte loads.  Jobs of lines
// of fft_wave_len lengths have at most one plane.
// ev (may be NULL): start and end events of the dispatch.
hipError_t dogk_fft_blur(const dog::LaunchArgs* args, const dog::FftJob* d_jobs, int n_jobs,
                         int logn, int vec, hipStream_t stream, hipEvent_t* ev);
}
