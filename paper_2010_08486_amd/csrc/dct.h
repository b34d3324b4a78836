// Transform-domain blur (dct.hip): one workgroup's job.  Not part of the
// public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dog_internal.h"

namespace dog {

// `lines` lines (even) starting at line0 of one length-N transform (N a
// power of two).  cols = 1: line l is column l of `in` (row-major, rows
// in_pitch floats apart, N rows); 0: line l is row l (N values).  Output
// line l is the row out + l * out_pitch.  Inverse jobs of the first inverse
// step scale the input by hline[line] * hpos[position].
struct DctJob {
    const float* in;         // NULL: the pixels of frame `frame` of the launch
    float* out;
    const float* hline;      // NULL: no scaling
    const float* hpos;
    const float2* tw;        // N/2 twiddles exp(-2 pi i t / N)
    const float2* post;      // N twiddles exp(-i pi k / (2N))
    int32_t in_pitch;
    int32_t out_pitch;
    int32_t N;
    int32_t logn;
    int32_t line0;
    int32_t lines;           // 2^(logp + 1), (lines / 2) * N <= 4096
    int32_t logp;
    int32_t cols;
    int32_t frame;
    int32_t pad_;
};

}  // namespace dog

extern "C" {
size_t dogk_dct_lds_bytes(int N, int lines);
// ev (may be NULL): start and end events of the dispatch.
hipError_t dogk_dct(const dog::LaunchArgs* args, const dog::DctJob* d_jobs, int n_jobs,
                    size_t lds_bytes, int inverse, hipStream_t stream, hipEvent_t* ev);
}
