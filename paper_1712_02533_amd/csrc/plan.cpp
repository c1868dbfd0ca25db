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
// Two schedules need more than "x[right] <- x[left] (.) x[right]" and are written as programs
// (pprs_scan_program): instructions over M elements plus scratch elements, executed in list
// order, each COMBINE dst <- a (.) b, MOVE dst <- a or CLEAR dst <- identity:
//  - Blelloch: algorithm "blelloch", the exclusive scan with the identity element: the
//    Brent-Kung up-sweep over the elements padded with identities to a power of two, the root
//    cleared to the identity (its total kept in a scratch element), then the down-sweep in which
//    each left child takes its parent's value and each right child the parent's value combined
//    with the left child's old value (parent (.) left: the order a non-commutative operator
//    needs; the listing writes left (.) parent). Exclusive value m is the inclusive value m - 1,
//    so the program ends by moving element m + 1 to m and the kept total to M - 1. A combine
//    with the identity is a copy (the identity costs nothing).
//  - reduce-then-scan (distributed chapter, algorithm "distributed_alternative_parallel"), P
//    workers with the chunks of the general strategy: every worker folds its chunk into a
//    scratch total without touching the elements, a Brent-Kung scan over the P totals (in place,
//    inclusive, so total I - 1 is what worker I needs), then every worker rescans its chunk
//    serially from that value: x[f] <- T_{I-1} (.) x[f], x[j] <- x[j-1] (.) x[j].
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

namespace {

// Program instructions (see the header comment).
struct Instr {
  int code, a, b, dst, level;
};

int workers_of(int M, int P) {
  if (P <= 0) P = (int)std::ceil(std::sqrt((double)M));
  return P > M ? M : P;
}

// Blelloch over M elements; scratch: M .. n2 - 1 padding (identity), n2 the kept total, n2 + 1
// the swap temporary. Levels: log2 n2 up-sweep steps, log2 n2 down-sweep steps.
std::vector<Instr> blelloch(int M, int* levels, int* n_elems) {
  std::vector<Instr> v;
  int lv = 0;
  if (M < 1) {
    *levels = 0;
    *n_elems = M;
    return v;
  }
  int n2 = 1;
  while (n2 < M) n2 *= 2;
  const int total = n2, tmp = n2 + 1;
  for (int d = 1; d < n2; d *= 2, ++lv)  // up-sweep
    for (int j = 2 * d - 1; j < n2; j += 2 * d) v.push_back({PPRS_SCAN_OP_COMBINE, j - d, j, j, lv});
  v.push_back({PPRS_SCAN_OP_MOVE, n2 - 1, -1, total, lv});
  v.push_back({PPRS_SCAN_OP_CLEAR, -1, -1, n2 - 1, lv});
  for (int d = n2 / 2; d >= 1; d /= 2, ++lv)  // down-sweep
    for (int j = 2 * d - 1; j < n2; j += 2 * d) {
      v.push_back({PPRS_SCAN_OP_MOVE, j - d, -1, tmp, lv});
      v.push_back({PPRS_SCAN_OP_MOVE, j, -1, j - d, lv});
      v.push_back({PPRS_SCAN_OP_COMBINE, j, tmp, j, lv});
    }
  for (int m = 0; m + 1 < M; ++m) v.push_back({PPRS_SCAN_OP_MOVE, m + 1, -1, m, lv});
  v.push_back({PPRS_SCAN_OP_MOVE, total, -1, M - 1, lv});
  *levels = lv;
  *n_elems = n2 + 2;
  return v;
}

// Reduce-then-scan over M elements with P workers; scratch M + I: worker I's total.
std::vector<Instr> reduce_then_scan(int M, int P, int* levels, int* n_elems) {
  std::vector<Instr> v;
  int lv = 0;
  *n_elems = M;
  if (M < 1) {
    *levels = 0;
    return v;
  }
  P = workers_of(M, P);
  *n_elems = M + P;
  std::vector<int> first(P + 1);
  for (int I = 0, at = 0; I <= P; ++I) {
    first[I] = at;
    at += M / P + (I < M % P ? 1 : 0);
  }
  const int kmax = M / P + (M % P ? 1 : 0);
  for (int I = 0; I < P; ++I) v.push_back({PPRS_SCAN_OP_MOVE, first[I], -1, M + I, lv});
  for (int st = 1; st < kmax; ++st, ++lv)  // reduce: each chunk folded into its total
    for (int I = 0; I < P; ++I)
      if (first[I] + st < first[I + 1])
        v.push_back({PPRS_SCAN_OP_COMBINE, M + I, first[I] + st, M + I, lv});
  std::vector<int> tot(P);
  for (int I = 0; I < P; ++I) tot[I] = M + I;
  std::vector<Op> bk;
  brent_kung(tot, bk, &lv);  // global scan over the totals
  for (const Op& o : bk) v.push_back({PPRS_SCAN_OP_COMBINE, o.left, o.right, o.right, o.level});
  for (int st = 0; st < kmax; ++st) {  // rescan, the chunks side by side
    bool any = false;
    for (int I = 0; I < P; ++I) {
      int j = first[I] + st;
      if (j >= first[I + 1]) continue;
      if (st == 0 && I == 0) continue;  // y_0 = x_0
      int left = st == 0 ? M + I - 1 : j - 1;
      v.push_back({PPRS_SCAN_OP_COMBINE, left, j, j, lv});
      any = true;
    }
    if (any) ++lv;
  }
  *levels = lv;
  return v;
}

std::vector<Instr> make_program(int kind, int M, int P, int* levels, int* n_elems) {
  if (kind == PPRS_SCAN_BLELLOCH) return blelloch(M, levels, n_elems);
  if (kind == PPRS_SCAN_REDUCE_THEN_SCAN) return reduce_then_scan(M, P, levels, n_elems);
  std::vector<Op> ops = make_plan(kind, M, P, levels);
  std::vector<Instr> v;
  for (const Op& o : ops) v.push_back({PPRS_SCAN_OP_COMBINE, o.left, o.right, o.right, o.level});
  *n_elems = M;
  return v;
}

// Registrations the program makes: combines whose operands are both non-identities (elements
// start as inputs, scratch as the identity; a combine with an identity copies the other).
int count_registrations(const std::vector<Instr>& v, int M, int n_elems) {
  std::vector<char> ident(n_elems, 1);
  for (int m = 0; m < M; ++m) ident[m] = 0;
  int n = 0;
  for (const Instr& x : v) {
    if (x.code == PPRS_SCAN_OP_COMBINE) {
      bool both = !ident[x.a] && !ident[x.b];
      n += both;
      ident[x.dst] = ident[x.a] && ident[x.b];
    } else if (x.code == PPRS_SCAN_OP_MOVE) {
      ident[x.dst] = ident[x.a];
    } else {
      ident[x.dst] = 1;
    }
  }
  return n;
}
}  // namespace

extern "C" pprs_status pprs_scan_program(int kind, int M, int P, int* prog, int cap,
                                         int* n_instr, int* n_levels, int* n_elems,
                                         int* n_reg) {
  if (M < 0 || P < 0 || kind < PPRS_SCAN_SEQUENTIAL || kind > PPRS_SCAN_REDUCE_THEN_SCAN ||
      !n_instr)
    return PPRS_EINVAL;
  int levels = 0, elems = M;
  std::vector<Instr> v = make_program(kind, M, P, &levels, &elems);
  *n_instr = (int)v.size();
  if (n_levels) *n_levels = levels;
  if (n_elems) *n_elems = elems;
  if (n_reg) *n_reg = count_registrations(v, M, elems);
  if ((int)v.size() > cap || (!prog && !v.empty())) return PPRS_EINVAL;
  for (size_t i = 0; i < v.size(); ++i) {
    prog[5 * i] = v[i].code;
    prog[5 * i + 1] = v[i].a;
    prog[5 * i + 2] = v[i].b;
    prog[5 * i + 3] = v[i].dst;
    prog[5 * i + 4] = v[i].level;
  }
  return PPRS_OK;
}

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
