// Host helpers that cut staging work into pieces of one workgroup each.
#pragma once
#include <algorithm>
#include <vector>

#include "types.hpp"

namespace bsm {

constexpr int kXposeBand = 64;             // rows of a transposition piece
constexpr int64_t kCopyPiece = 1 << 16;    // elements of a copy piece
constexpr int64_t kPermPiece = 1 << 16;    // elements of a permutation piece

// Transpose a rows x cols row-major block at src into the cols x rows row-major block at dst.
inline void push_transpose(std::vector<XposeBlock>& t, int64_t src, int64_t dst, int32_t rows,
                           int32_t cols) {
  for (int32_t r0 = 0; r0 < rows; r0 += kXposeBand)
    t.push_back(XposeBlock{src + int64_t(r0) * cols, dst + r0, std::min(kXposeBand, rows - r0),
                           cols, cols, rows});
}

// Copy n contiguous elements.
inline void push_copy(std::vector<CopyBlock>& t, int64_t src, int64_t dst, int64_t n) {
  for (int64_t e = 0; e < n; e += kCopyPiece)
    t.push_back(CopyBlock{src + e, dst + e, std::min(kCopyPiece, n - e)});
}

}  // namespace bsm
