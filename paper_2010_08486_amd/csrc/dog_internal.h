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

namespace dog {

// One frame of a launch.
struct FrameDesc {
    const float* src;        // input frame (device)
    float* T;                // n_g transposed planes of pass 1
    float* L;                // n_g transposed planes of pass 2
    float* Ddbg;             // optional: k transposed DoG planes written by the NMS kernel
    long long src_stride;    // elements between input rows
    long long pitch;         // elements between rows of a transposed plane
    int H, W;
    int ladder;              // index into the ladder table
    int frame_id;            // value written into candidate records
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

// A unit of work of one kernel: one (frame, plane) for the blur passes or one
// frame for the local-maximum kernel, restricted to the column blocks
// [cb0, cb0 + n_cb) and tiled into n_cb x n_band tiles.
struct WorkUnit {
    int frame;
    int plane;
    int cb0;           // first column block of this slice
    int n_cb;          // column blocks in this slice
    int n_band;        // row bands
    int first_tile;    // prefix sum of tiles over the preceding units of the same list
    int pad_[2];
};

#define DOG_NXCD 8     // accelerator complex dies (each with its own L2)

// One kernel's work split into DOG_NXCD lists, one per XCD: list c holds the
// column slices meant to stay in XCD c's L2 and is drained first by the
// workgroups dispatched to XCD c (workgroup id mod 8); idle workgroups then
// steal from the other lists.
struct Queue {
    const WorkUnit* units;     // all lists back to back
    int off[DOG_NXCD];         // first unit of list c
    int n[DOG_NXCD];           // units in list c
    int total[DOG_NXCD];       // tiles in list c
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

// Tile counters of the three persistent kernels, one per XCD list.  Block 0
// of each kernel clears the counters of the kernel two steps ahead in the
// launch sequence (pass 1 -> local maxima, pass 2 -> pass 1, local maxima ->
// pass 2), which are never in use at that time.
struct Counters {
    uint32_t c[3][DOG_NXCD];
};

// Arguments of one launch sequence (all pointers are device pointers).
struct LaunchArgs {
    const FrameDesc* frames;
    const LadderDesc* ladders;
    const float* weights;
    const Queue* queues;        // [3]: pass 1, pass 2, local maxima
    Counters* counters;
    CandHeader* cand;           // header; records at (CandRec*)(cand + 1)
    uint32_t cap;               // record capacity
    int pad_;
};


}  // namespace dog
