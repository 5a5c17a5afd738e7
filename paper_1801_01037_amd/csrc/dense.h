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

// A general gate on k <= 5 qubits of a small register (one work-group per
// setting of the other bits; used below 9 qubits, where k_dense5 has too few
// columns).
struct SmallUArgs {
    void *psi;
    const void *mat;     // 2^k x 2^k complex, row major, FP64 (re, im)
    uint64_t omask;      // the other index bits
    uint64_t ngroups;    // 2^(n-k)
    uint64_t off[32];    // index offset of local combination c (q_0 = bit 0 of c)
    int32_t dim;         // 2^k
};
hipError_t launch_unitary_small(const SmallUArgs &a, bool c64, hipStream_t st);

}  // namespace svk
