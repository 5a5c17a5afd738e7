// Dense 5-qubit block pass (SV_FUSE_DENSE).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace svk {

struct DenseArgs {
    void *psi;
    const void *mat;     // the block's real 64x64 form [[Re M, -Im M], [Im M, Re M]],
                         // row major, double (complex128) or float (complex64)
    uint64_t bmask;      // the 5 index bits of the block
    uint64_t omask;      // the other index bits of the register
    uint64_t ncols;      // 2^(n-5) columns; a multiple of 16 (n >= 9)
};

// Requires n >= 9 (at least 16 columns).
hipError_t launch_dense5(const DenseArgs &a, bool c64, hipStream_t st);

}  // namespace svk
