// Range checks of the counting sort that builds the fibre orderings, shared
// by its kernels and by a host test (no HIP types here).
//
// A counting sort scatters entry p to ptr[slot] + (its rank among the
// slot's entries). If the exclusive scan of the slot counts were wrong, that
// position could fall outside the output; these predicates let the kernels
// skip such a write and raise a flag instead, which the host turns into an
// error status.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define TK_HD __host__ __device__
#else
#define TK_HD
#endif

namespace tk {

// Bit of the preparation flags word set when an ordering fails its checks.
constexpr int32_t kFlagOrderCheck = 4;

// The scan of the slot counts must end at the number of entries sorted.
TK_HD inline bool order_total_ok(int32_t scanned_total, int64_t nnz) { return (int64_t)scanned_total == nnz; }

// Entry position pos of a slot whose entries occupy [begin, end), inside an
// output of nnz entries.
TK_HD inline bool order_pos_ok(int64_t pos, int32_t begin, int32_t end, int64_t nnz) {
    return begin >= 0 && begin <= end && (int64_t)end <= nnz && pos >= begin && pos < end;
}

// Status of a preparation from its flags word: 1 = a coordinate out of range,
// 2 = a non-finite value, kFlagOrderCheck = an ordering failed its checks.
// Returns 0 (no error) or -2 (index), -3 (value), -6 (device) in the
// library's status numbering.
TK_HD inline int prep_status(int32_t flags) {
    if (flags & 1) return -2;
    if (flags & 2) return -3;
    if (flags & kFlagOrderCheck) return -6;
    return 0;
}

}  // namespace tk
