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
//  - general strategy (distributed chapter, algorithm "distributed_parallel") with P workers:
//    worker I holds K_I consecutive elements (one more for the first M mod P workers). Local
//    stage one: a serial scan inside every chunk, the chunks side by side. Global stage: a
//    Brent-Kung scan over the P chunk ends, in place, so the end of chunk I-1 holds the total
//    of everything before chunk I. Local stage two: every other element of chunk I > 0 takes
//    that end as its left operand (the chunk's own end is final after the global stage).
#include <cmath>
#include <vector>
#include "../../include/pprs.h"

namespace {
struct Op {
  int left, right, level;
};

// Brent-Kung over the elements idx[0..n): ops on the listed indices, levels from *lv on.
void brent_kung(const std::vector<int>& idx, std::vector<Op>& ops, int* lv) {
  const int n = (int)idx.size();
  for (int d = 1; d < n; d *= 2) {
    bool any = false;
    for (int j = 2 * d - 1; j < n; j += 2 * d) {
      ops.push_back({idx[j - d], idx[j], *lv});
      any = true;
    }
    if (any) ++*lv;
  }
  int top = 1;
  while (top * 2 < n) top *= 2;
  for (int d = top; d >= 1; d /= 2) {
    bool any = false;
    for (int j = 3 * d - 1; j < n; j += 2 * d) {
      ops.push_back({idx[j - d], idx[j], *lv});
      any = true;
    }
    if (any) ++*lv;
  }
}

std::vector<Op> make_plan(int kind, int M, int P, int* levels) {
  std::vector<Op> ops;
  int lv = 0;
  if (kind == PPRS_SCAN_GENERAL) {
    if (M > 0) {
      if (P <= 0) P = (int)std::ceil(std::sqrt((double)M));
      if (P > M) P = M;
      std::vector<int> first(P + 1);
      for (int I = 0, at = 0; I <= P; ++I) {
        first[I] = at;
        at += M / P + (I < M % P ? 1 : 0);
      }
      const int kmax = M / P + (M % P ? 1 : 0);
      for (int st = 1; st < kmax; ++st, ++lv)  // local stage one, chunks side by side
        for (int I = 0; I < P; ++I)
          if (first[I] + st < first[I + 1]) ops.push_back({first[I] + st - 1, first[I] + st, lv});
      std::vector<int> ends(P);
      for (int I = 0; I < P; ++I) ends[I] = first[I + 1] - 1;
      brent_kung(ends, ops, &lv);  // global stage
      bool any = false;
      for (int I = 1; I < P; ++I)  // local stage two
        for (int j = first[I]; j < first[I + 1] - 1; ++j) {
          ops.push_back({first[I] - 1, j, lv});
          any = true;
        }
      if (any) ++lv;
    }
  } else if (kind == PPRS_SCAN_SEQUENTIAL) {
    for (int m = 1; m < M; ++m) ops.push_back({m - 1, m, lv++});
  } else if (kind == PPRS_SCAN_KOGGE_STONE) {
    for (int d = 1; d < M; d *= 2, ++lv)
      for (int j = M - 1; j >= d; --j) ops.push_back({j - d, j, lv});
  } else if (kind == PPRS_SCAN_SKLANSKY) {
    for (int d = 1; d < M; d *= 2, ++lv)
      for (int j = d - 1; j < M; j += 2 * d)
        for (int k = 0; k < d && j + k + 1 < M; ++k) ops.push_back({j, j + k + 1, lv});
  } else {
    std::vector<int> all(M > 0 ? M : 0);
    for (int j = 0; j < M; ++j) all[j] = j;
    brent_kung(all, ops, &lv);
  }
  *levels = lv;
  return ops;
}
}  // namespace

extern "C" pprs_status pprs_scan_plan_p(int kind, int M, int P, int* ops, int cap, int* n_ops,
                                        int* n_levels) {
  if (M < 0 || P < 0 || kind < PPRS_SCAN_SEQUENTIAL || kind > PPRS_SCAN_GENERAL || !n_ops)
    return PPRS_EINVAL;
  int levels = 0;
  std::vector<Op> v = make_plan(kind, M, P, &levels);
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

extern "C" pprs_status pprs_scan_plan(int kind, int M, int* ops, int cap, int* n_ops,
                                      int* n_levels) {
  return pprs_scan_plan_p(kind, M, 0, ops, cap, n_ops, n_levels);
}
