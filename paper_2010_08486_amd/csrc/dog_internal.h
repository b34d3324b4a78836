// Internal structures shared by the host runtime and the HIP kernels of the
// Difference-of-Gaussians detector.  Not part of the public C ABI.
//
// Data layout in device memory (one frame of H rows x W columns, n_g = k+1
// Gaussian planes, k DoG planes):
//   * input X           : H x W fp32, row stride src_stride (elements).
//   * T planes (pass 1) : n_g planes, each stored TRANSPOSED as W rows of
//                         `pitch` floats (pitch >= H, multiple of 64):
//                         T_p[x * pitch + y] = sum_j w_p[j] X[refl(y+j)][x].
//   * L planes (pass 2) : same transposed layout,
//                         L_p[x * pitch + y] = sum_j w_p[j] T_p[refl(x+j)*pitch + y].
//   * DoG planes are never stored: the local-maximum kernel forms
//     D_i = sigma_i * (L_i - L_{i+1}) in registers.
// Both blur passes therefore walk down the columns of their input, with lanes
// across a row (coalesced) and the reflection in the walking direction, where
// it is wave-uniform.
#pragma once
#include <stdint.h>

#define DOG_MAX_GAUSS 64              // n_g limit (k <= 63 DoG planes)
#define DOG_WPAD 16                   // per-plane weight vectors padded to a multiple of this
#define DOG_NMS_COLS 62               // output columns per wave of the local-maximum kernel
#define DOG_FFT_MERGED 4              // blur kernels with transform jobs of lines of 2^7 .. 2^10

namespace dog {

// One frame of a launch.
struct FrameDesc {
    const float* src;        // input frame (device)
    float* T;                // n_g transposed planes of pass 1
    float* L;                // n_g transposed planes of pass 2
    float* Ddbg;             // optional: k transposed DoG planes written by the NMS kernel
    const int* rows1;        // pass 1: byte offset of input row refl(t, H), t = -pad .. H+pad-1
    const int* rows2;        // pass 2: byte offset of T row refl(t, W), t = -pad .. W+pad-1
    long long src_stride;    // elements between input rows
    long long pitch;         // elements between rows of a transposed plane
    int H, W;
    int ladder;              // index into the ladder table
    int frame_id;            // value written into candidate records
    int pad;                 // rows of reflection on each side of the row tables
    int pad_;
};

// A sigma ladder after planning (Sec. 4 Eq. 1 in geometric form).
struct LadderDesc {
    int n_g;                      // Gaussian planes (k+1)
    int pad_;
    float thr;                    // largest float <= threshold: D > thr (fp32) <=> (double)D > threshold
    float pad2_;
    int r[DOG_MAX_GAUSS];         // kernel radii
    int woff[DOG_MAX_GAUSS];      // offset of plane p's weights in the weight array
    float sigma[DOG_MAX_GAUSS];   // sigma_p rounded to fp32 (DoG scale factor)
};

#define DOG_NXCD 8     // accelerator complex dies (each with its own L2)

// One workgroup's tile: column block cb and row band of plane `plane` of
// frame `frame` (plane unused by the local-maximum kernel).  Each kernel is
// launched with one workgroup per tile and reads its tile from a host-built
// table indexed by the workgroup id; the table lists the tiles widest kernel
// first and interleaves XCD-local column slices so that workgroup b, which
// the dispatcher places on XCD b mod 8, works on that XCD's slice.
struct Tile {
    uint16_t frame;
    uint8_t plane;
    uint8_t n_planes;   // staged blur: planes plane, plane-1, ..., in turn (0: one)
    uint16_t cb;
    uint16_t band;
};

// Candidate record written by the local-maximum kernel.
struct CandRec {
    int32_t frame;
    int32_t y;
    int32_t x;
    int32_t scale;
    float response;
};

// Header of the candidate buffer; records follow at byte offset 16.
struct CandHeader {
    uint32_t count;       // number of candidates found (may exceed cap)
    uint32_t pad_[3];
};

struct FftJob;   // transform-domain job (dct.h)

// Arguments of one launch sequence (all pointers are device pointers).
struct LaunchArgs {
    const FrameDesc* frames;    // frame table, or NULL: the one frame is f0
    const LadderDesc* ladders;
    const float* weights;
    const Tile* tiles1;         // pass 1, one per workgroup
    const Tile* tiles2;         // pass 2
    const Tile* tiles3;         // local maxima
    CandHeader* cand;           // header; records at (CandRec*)(cand + 1)
    CandRec* host_recs;         // pinned host copy of the first n_host records
    uint32_t* host_ends;        // pinned host: per local-maximum workgroup, the
                                // end of its record range (the count is the max)
    uint32_t cap;               // record capacity
    uint32_t n_host;
    int n1, n2, n3;             // tiles of each kernel
    int pad_;
    FrameDesc f0;               // the frame of a one-frame launch (frames == NULL)
    const FftJob* fft_jobs[2];  // transform-domain jobs run by blur pass 1 / 2
    int n_fft[2];               // their count (a multiple of DOG_NXCD), or 0
};

// The transform-domain blur's launches of a sequence: for pass 1 (along y)
// and pass 2 (along x), one launch per line length (log2 N = 6..11) with its
// job table (device) and count, and whether every job's input allows
// 8-byte loads; or, when a pass's jobs all have one line length the blur
// kernels can take, none (the jobs run in the blur pass's launch).
struct FftLaunch {
    const void* jobs[2][6];
    int n[2][6];
    int vec[2];
    int merged_logn[2];         // > 0: the pass's jobs run in the blur launch (LaunchArgs)
    int total(int pass) const
    {
        int t = 0;
        for (int i = 0; i < 6; ++i)
            t += n[pass][i];
        return t;
    }
};

}  // namespace dog
