// Scan schedules over M elements (host only, no HIP). An op (left, right, level) means
// x[right] <- x[left] (.) x[right]; ops sharing a level are mutually independent.
//  - sequential: algorithm "serial" of the Prefix sum chapter: y_m = y_{m-1} (.) x_m.
//  - Brent-Kung: algorithm "brent_kung": up-sweep x_j <- x_{j-d} (.) x_j for j = 2d-1, 4d-1,
//    ... (d = 1, 2, 4, ...), then down-sweep x_j <- x_{j-d} (.) x_j for j = 3d-1, 5d-1, ...
//    with d halving from the largest power of two below M. Valid for any M (the paper's
//    listing assumes a power of two; its up-sweep indices are read in this standard form).
//  - Kogge-Stone: algorithm "kogge_stone": for d = 1, 2, 4, ...: x_j <- x_{j-d} (.) x_j for
//    every j >= d with the previous step's values (the listing's lower bound of j is read as
//    d = 2^i). A level is listed right to left, so each op reads its left operand before the
//    op that rewrites it.
//  - Sklansky: algorithm "sklansky": for d = 1, 2, 4, ...: in each block of 2d elements the
//    upper d take the last element of the lower d as left operand (its value is final for the
//    block, and nothing in the level rewrites it).
#include <vector>
#include "../../include/pprs.h"

namespace {
struct Op {
  int left, right, level;
};

std::vector<Op> make_plan(int kind, int M, int* levels) {
  std::vector<Op> ops;
  int lv = 0;
  if (kind == PPRS_SCAN_SEQUENTIAL) {
    for (int m = 1; m < M; ++m) ops.push_back({m - 1, m, lv++});
  } else if (kind == PPRS_SCAN_KOGGE_STONE) {
    for (int d = 1; d < M; d *= 2, ++lv)
      for (int j = M - 1; j >= d; --j) ops.push_back({j - d, j, lv});
  } else if (kind == PPRS_SCAN_SKLANSKY) {
    for (int d = 1; d < M; d *= 2, ++lv)
      for (int j = d - 1; j < M; j += 2 * d)
        for (int k = 0; k < d && j + k + 1 < M; ++k) ops.push_back({j, j + k + 1, lv});
  } else {
    for (int d = 1; d < M; d *= 2) {
      bool any = false;
      for (int j = 2 * d - 1; j < M; j += 2 * d) {
        ops.push_back({j - d, j, lv});
        any = true;
      }
      if (any) ++lv;
    }
    int top = 1;
    while (top * 2 < M) top *= 2;
    for (int d = top; d >= 1; d /= 2) {
      bool any = false;
      for (int j = 3 * d - 1; j < M; j += 2 * d) {
        ops.push_back({j - d, j, lv});
        any = true;
      }
      if (any) ++lv;
    }
  }
  *levels = lv;
  return ops;
}
}  // namespace

extern "C" pprs_status pprs_scan_plan(int kind, int M, int* ops, int cap, int* n_ops,
                                      int* n_levels) {
  if (M < 0 || kind < PPRS_SCAN_SEQUENTIAL || kind > PPRS_SCAN_SKLANSKY || !n_ops)
    return PPRS_EINVAL;
  int levels = 0;
  std::vector<Op> v = make_plan(kind, M, &levels);
  *n_ops = (int)v.size();
  if (n_levels) *n_levels = levels;
  if ((int)v.size() > cap || (!ops && !v.empty())) return PPRS_EINVAL;
  for (size_t i = 0; i < v.size(); ++i) {
    ops[3 * i] = v[i].left;
    ops[3 * i + 1] = v[i].right;
    ops[3 * i + 2] = v[i].level;
  }
  return PPRS_OK;
}
