// Device-side overlap pruning and radius histogram (prune_device.hip): launch
// arguments and the per-frame output layout.  Not part of the public C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dog_internal.h"

namespace dog {

enum PruneStatus : int32_t {
    kPruneDone = 1,           // survivors and histogram written
    kPruneTooManyBlobs = 2,   // more blobs than one workgroup holds: host step instead
    kPruneTooManyPairs = 3,   // more touching pairs than the workgroup holds: host step
    kPruneListOverflow = 4,   // the candidate list overflowed its buffer: host step
    kPruneBadRecord = 5,      // a record outside 0 <= y, x < 32768, 0 <= scale < k
};

// Output of one frame: this header, then up to max_blobs dog_blob records
// (survivors in (y, x, scale) order).
struct PruneHead {
    int32_t status;
    uint32_t n_raw;                 // blobs of the frame before pruning
    uint32_t n_out;                 // survivors
    uint32_t pad_;
    uint32_t hist[DOG_MAX_GAUSS];   // survivors per radius bin (k bins)
};

struct PruneArgs {
    const CandHeader* cand;   // candidate list header (count), or NULL: n_direct records
    const void* recs;         // CandRec records with frame ids, or (blob_in) dog_blob records
    uint32_t cap;             // records the list holds
    uint32_t n_direct;        // record count when cand is NULL
    const double* sig64;      // FP64 sigmas of the ladder's k+1 planes (device)
    double sig_max;           // largest sigma of the k DoG scales
    double overlap;           // >= 1: no pruning
    int32_t k;                // DoG scales = histogram bins
    int32_t coalesce;
    int32_t blob_in;
    uint32_t max_blobs;       // blobs one workgroup holds (power of two, <= 4096)
    uint32_t max_pairs;       // touching pairs one workgroup holds
    uint32_t pad_;
    char* out;                // frame f's output at out + f * out_stride
    uint64_t out_stride;
};

}  // namespace dog

extern "C" {
size_t dogk_prune_lds_bytes(uint32_t max_blobs, uint32_t max_pairs);
hipError_t dogk_prune(const dog::PruneArgs* args, int n_frames, hipStream_t stream);
}
