// LDS slot of a tile element, shared by the pass packer (host) and the tile
// kernel (device).
//
// The bits of element index j at positions >= B are folded into its low B
// bits through fixed B-bit columns: a linear map over GF(2), so
// sw(a ^ b) = sw(a) ^ sw(b), and a bijection on [0, 2^t) (the high bits stay).
// An operator's group members differ in the bits of its positions; when those
// include low positions, the lanes of a wave spread over higher bits, and
// without the fold they would meet in few LDS banks.  B covers one row of
// 32 four-byte banks (16 complex64 or 8 complex128 elements).  The columns
// were chosen by a search minimising the simulated bank conflicts of the
// operators the pass planner emits for deep Pauli-exponential circuits.
#pragma once

namespace qs {

constexpr int kSwzB64 = 4;    // complex64
constexpr int kSwzB128 = 3;   // complex128
constexpr int kSwzCols = 10;
constexpr int kSwzCols64[kSwzCols] = {15, 11, 6, 1, 1, 3, 10, 1, 12, 5};
constexpr int kSwzCols128[kSwzCols] = {7, 6, 3, 1, 1, 2, 5, 1, 6, 3};

// QSIM_LDS_FOLD selects the fold: 0 none, 1 the plain fold (bit p >= B lands
// on bit p mod B), 2 the searched columns (the default: 1-3% faster than the
// plain fold on the 21-qubit benchmark circuit).
#ifndef QSIM_LDS_FOLD
#define QSIM_LDS_FOLD 2
#endif

// elem_bytes: 8 (complex64) or 16 (complex128)
constexpr int lds_slot(int elem_bytes, int j) {
    const int B = elem_bytes == 8 ? kSwzB64 : kSwzB128;
#if QSIM_LDS_FOLD == 0
    (void)B;
    return j;
#elif QSIM_LDS_FOLD == 1
    int acc = 0;
    for (int h = j >> B; h; h >>= B) acc ^= h;
    return j ^ (acc & ((1 << B) - 1));
#else
    const int *cols = elem_bytes == 8 ? kSwzCols64 : kSwzCols128;
    int acc = 0;
    for (int i = 0; i < kSwzCols; i++)
        if ((j >> (B + i)) & 1) acc ^= cols[i];
    return j ^ acc;
#endif
}

}  // namespace qs
