// validate.cpp -- BLAS argument checks and operand-overlap tests of single
// calls and grouped batches.  Host code only, free of HIP: no check here
// touches a device.
#include <stdint.h>

#include <algorithm>
#include <iterator>
#include <string>
#include <vector>

#include "host_common.hpp"

namespace mgemm {

int trans_code(char t) {
    if (t == 'N' || t == 'n') return 0;
    if (t == 'T' || t == 't' || t == 'C' || t == 'c') return 1;
    return -1;
}

static int64_t max1(int64_t v) { return v > 1 ? v : 1; }

// Byte range [lo, hi) touched by the referenced part of a stored array
// (rows, cols >= 1).  Computed in 128 bits and clamped to the address
// space, so that no leading dimension a caller passes overflows it.
static void extent(const void* p, int64_t rows, int64_t cols, int64_t ld, uintptr_t& lo,
                   uintptr_t& hi) {
    lo = (uintptr_t)p;
    const unsigned __int128 bytes =
        ((unsigned __int128)(uint64_t)(cols - 1) * (uint64_t)ld + (uint64_t)rows) * sizeof(float);
    const unsigned __int128 end = (unsigned __int128)lo + bytes;
    hi = end > (unsigned __int128)UINTPTR_MAX ? UINTPTR_MAX : (uintptr_t)end;
}

int validate(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
             const float* A, int64_t lda, const float* B, int64_t ldb, float beta,
             const float* C, int64_t ldc, std::string& why) {
    const int ta = trans_code(transA), tb = trans_code(transB);
    if (ta < 0) { why = "transA must be N, T or C"; return -1; }
    if (tb < 0) { why = "transB must be N, T or C"; return -2; }
    if (M < 0) { why = "M < 0"; return -3; }
    if (N < 0) { why = "N < 0"; return -4; }
    if (K < 0) { why = "K < 0"; return -5; }
    const int64_t rows_a = ta ? K : M, rows_b = tb ? N : K;
    const bool reads_ab = alpha != 0.0f && K > 0 && M > 0 && N > 0;
    if (reads_ab && A == nullptr) { why = "A is NULL"; return -7; }
    if (lda < max1(rows_a)) { why = "lda < max(1, stored rows of A)"; return -8; }
    if (reads_ab && B == nullptr) { why = "B is NULL"; return -9; }
    if (ldb < max1(rows_b)) { why = "ldb < max(1, stored rows of B)"; return -10; }
    if (M > 0 && N > 0 && C == nullptr) { why = "C is NULL"; return -12; }
    if (ldc < max1(M)) { why = "ldc < max(1, M)"; return -13; }
    (void)beta;
    return 0;
}

// C must not overlap the referenced part of A or B (the kernels read A and
// B while other work-groups write C).
bool overlaps(int ta, int tb, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
              int64_t lda, const float* B, int64_t ldb, const float* C, int64_t ldc) {
    if (alpha == 0.0f || K == 0 || M == 0 || N == 0) return false;
    uintptr_t clo, chi, lo, hi;
    extent(C, M, N, ldc, clo, chi);
    extent(A, ta ? K : M, ta ? M : K, lda, lo, hi);
    if (lo < chi && clo < hi) return true;
    extent(B, tb ? N : K, tb ? K : N, ldb, lo, hi);
    return lo < chi && clo < hi;
}

Extent extent_of(const void* p, int64_t rows, int64_t cols, int64_t ld, int64_t owner) {
    Extent e{};
    extent(p, rows, cols, ld, e.lo, e.hi);
    e.owner = owner;
    return e;
}

int64_t batch_alias(std::vector<Extent> cs, const std::vector<Extent>& ab, int* kind) {
    std::sort(cs.begin(), cs.end(), [](const Extent& a, const Extent& b) { return a.lo < b.lo; });
    for (size_t k = 1; k < cs.size(); ++k)
        if (cs[k].lo < cs[k - 1].hi) {
            if (kind) *kind = 1;
            return cs[k].owner;
        }
    for (const Extent& x : ab) {
        // The C extent with the largest start below x's end is the only one
        // that can overlap x (the C extents are disjoint and sorted).
        auto it = std::lower_bound(cs.begin(), cs.end(), x.hi,
                                   [](const Extent& c, uintptr_t v) { return c.lo < v; });
        if (it != cs.begin() && std::prev(it)->hi > x.lo) {
            if (kind) *kind = 2;
            return std::prev(it)->owner;
        }
    }
    if (kind) *kind = 0;
    return -1;
}

}  // namespace mgemm
