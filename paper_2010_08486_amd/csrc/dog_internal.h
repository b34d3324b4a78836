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

// A unit of blur work: one (frame, plane), tiled into column blocks x row bands.
// For the local-maximum kernel the plane field is unused (one unit per frame).
struct WorkUnit {
    int frame;
    int plane;
    int n_cb;          // column blocks
    int n_band;        // row bands
    int first_tile;    // prefix sum of tiles over the preceding units
    int pad_[3];
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

// Work counters of the three persistent kernels.  Each kernel clears the
// counter of the kernel two steps ahead in the launch sequence; see kernels.hip.
struct Counters {
    uint32_t pass1;
    uint32_t pass2;
    uint32_t nms;
    uint32_t pad_;
};

// Arguments of one launch sequence (all pointers are device pointers).
struct LaunchArgs {
    const FrameDesc* frames;
    const LadderDesc* ladders;
    const float* weights;
    const WorkUnit* units1;     // pass 1 units
    const WorkUnit* units2;     // pass 2 units
    const WorkUnit* units3;     // local-maximum units (one per frame)
    Counters* counters;
    CandHeader* cand;           // header; records at (CandRec*)(cand + 1)
    int n_units1, n_units2, n_units3;
    int total1, total2, total3; // tiles of each kernel
    uint32_t cap;               // record capacity
    int pad_;
};

// Kernel tile geometry (compile-time variants, chosen per size class).
struct Geometry {
    int S;           // outputs per thread along the walking direction
    int NW;          // waves per workgroup
    int BI;          // strips per wave per tile
    int band() const { return S * NW * BI; }
};

}  // namespace dog
