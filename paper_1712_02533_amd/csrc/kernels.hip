// HIP kernels of libpprs for gfx950 (MI355X): 64-wide wavefronts, LDS-staged stencils,
// FP32 arithmetic with FP64 reductions, deterministic fixed-order sums.
//
// Per-step kernels (one "step" advances every active registration by one phase):
//   k_plan     - builds per-kind item lists from the slot phases (one workgroup)
//   k_grad     - applies the accepted step and computes the gradient G; in the same launch,
//                the bilinear prolongation of a finished level's u to the next level
//   k_energy_step - energies at the step sizes of a line-search pass, and the start energy
//                of a level, in one launch
//   k_smooth   - metric solve d = (S1^-1 (x) S1^-1) G, one direction per launch
//   k_*_fin    - per-slot finalisers, launched after a pass: sum the pass's FP64 tile partials
//                in tile order and advance the slot's state (the kernel boundary orders them
//                after every tile; no fences or tickets inside a pass)
#include <hip/hip_runtime.h>
#include <math.h>
#include "pprs_internal.h"
#include "kernels.h"

// minimum waves per SIMD the hot kernels are compiled for (register budget 512 / value)
#define LB_ENERGY 4
#define LB_GRAD 4
#define LB_SMOOTH 4

#define FLAG_NONCONV 1
#define FLAG_NAN 2


// ------------------------------------------------------------------------------------------
// Helpers

__device__ __forceinline__ int lvl_n(int l) { return (1 << l) + 1; }

typedef float f32x2u __attribute__((ext_vector_type(2), aligned(4)));

// Global-address-space access. Pointers read out of the batch descriptor are generic to the
// compiler, which then emits flat loads: those also count against the LDS counter, so every
// wait for a gather drained the LDS traffic too. All device buffers here are global memory.
#define GAS __attribute__((address_space(1)))
__device__ __forceinline__ float gld(const float* p, size_t i) {
  return ((const GAS float*)p)[i];
}
__device__ __forceinline__ void gst(float* p, size_t i, float v) { ((GAS float*)p)[i] = v; }

// A block-uniform pointer moved to scalar registers, so loads through it can take a scalar
// base with a 32-bit per-lane offset (the compiler does not always see that a pointer read
// out of the batch descriptor is uniform).
template <class P>
__device__ __forceinline__ P* uni(P* p) {
  unsigned long long v = (unsigned long long)p;
  unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (P*)(((unsigned long long)hi << 32) | lo);
}
// floor(x) converted to int in one instruction (v_cvt_flr_i32_f32; 0 for NaN like a plain
// conversion).
__device__ __forceinline__ int cvt_flr(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
// a * b + c on 24-bit a and b (v_mad_i32_i24): full rate, where a 32-bit product is not.
__device__ __forceinline__ int mad24(int a, int b, int c) {
  int r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
// The two corners of a row at byte offset o of g in one 8-byte load (rows are only 4-byte
// aligned). A 32-bit offset lets a block-uniform g stay a scalar base.
__device__ __forceinline__ f32x2u ld_pair(const float* g, unsigned o) {
  return *reinterpret_cast<const GAS f32x2u*>((const GAS char*)g + o);
}

// One float at byte offset o of a block-uniform base (scalar base + 32-bit lane offset: no
// 64-bit address arithmetic per access). Every buffer a kernel addresses this way is under
// 4 GiB from its base.
__device__ __forceinline__ float ldo(const float* g, unsigned o) {
  return *reinterpret_cast<const GAS float*>((const GAS char*)g + o);
}
__device__ __forceinline__ void sto(float* g, unsigned o, float v) {
  *reinterpret_cast<GAS float*>((GAS char*)g + o) = v;
}

// A node's bilinear coefficients (c0 v, c1 v(+x) - v, c2 v(+y) - v, c3 the cross difference)
// from the coefficient pyramid, at byte offset o of the frame's first record.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 ld_coef(const float* C, unsigned o) {
  return *reinterpret_cast<const GAS f32x4*>((const GAS char*)C + o);
}

// Clamped bilinear sample of nodal g (n x n) at column bi + tx, row ai + ty (cells).
// Returns value; writes the gradient in domain units when grad is true (zero across a
// coordinate whose position lies outside the level). The position is clamped to the level
// first and the cell index to n - 2, so a position on or beyond the far edge is cell n - 2 at
// fraction 1; inside, the fraction is tx - floor(tx).
template <bool GRAD>
__device__ __forceinline__ float sample_bil(const float* __restrict__ g, int n, int bi,
                                            float tx, int ai, float ty, float inv_h,
                                            float* gx, float* gy) {
  float cx = __builtin_amdgcn_fmed3f(tx, (float)(-bi), (float)(n - 1 - bi));
  float cy = __builtin_amdgcn_fmed3f(ty, (float)(-ai), (float)(n - 1 - ai));
  int ix = min(cvt_flr(cx), n - 2 - bi), iy = min(cvt_flr(cy), n - 2 - ai);
  float fx = cx - (float)ix, fy = cy - (float)iy;
  unsigned o = (unsigned)mad24(ai + iy, n, bi + ix) << 2;  // both indexes in [0, n - 2]
  f32x2u r0 = ld_pair(g, o);
  f32x2u r1 = ld_pair(g, o + ((unsigned)n << 2));
  float v00 = r0.x, v01 = r0.y, v10 = r1.x, v11 = r1.y;
  float top = fmaf(fx, v01 - v00, v00);
  float bot = fmaf(fx, v11 - v10, v10);
  if (GRAD) {
    *gx = cx != tx ? 0.f : fmaf(fy, (v11 - v10) - (v01 - v00), v01 - v00) * inv_h;
    *gy = cy != ty ? 0.f : (bot - top) * inv_h;
  }
  return fmaf(fy, bot - top, top);
}

// Clamped bilinear sample with its gradient (domain units) for the gradient pass, at (tx, ty)
// cells from the node whose byte offset is base4 in the plain pyramid (bounds relative to that
// node as in sample_cells; T0 the frame, T1 the frame one row down, both scalar bases; n4 the
// row pitch in bytes). The gradient pass reads the plain pyramid, not the coefficient records:
// its four samples per element gain less from the shorter arithmetic than they lose to the
// records' fourfold footprint in the caches. The cell index is clamped to the last cell (ixmax, iymax relative to the
// node), so a position on the far edge is the last cell at fraction 1 and its gradient that
// cell's slope; across a coordinate clamped to the level the gradient is zero.
__device__ __forceinline__ float sample_grad(const float* T0, const float* T1, unsigned n4,
                                             unsigned base4, float lox, float hix, float loy,
                                             float hiy, int ixmax, int iymax, float tx,
                                             float ty, float inv_h, float* gx, float* gy) {
  float cx = __builtin_amdgcn_fmed3f(tx, lox, hix);
  float cy = __builtin_amdgcn_fmed3f(ty, loy, hiy);
  int ix = min(cvt_flr(cx), ixmax), iy = min(cvt_flr(cy), iymax);
  float fx = cx - (float)ix, fy = cy - (float)iy;
  unsigned o = (unsigned)mad24(iy, (int)n4, (int)(base4 + ((unsigned)ix << 2)));
  f32x2u r0 = ld_pair(T0, o);
  f32x2u r1 = ld_pair(T1, o);
  float d0 = r0.y - r0.x, d1 = r1.y - r1.x;
  float top = fmaf(fx, d0, r0.x);
  float bot = fmaf(fx, d1, r1.x);
  *gx = cx != tx ? 0.f : fmaf(fy, d1 - d0, d0) * inv_h;
  *gy = cy != ty ? 0.f : (bot - top) * inv_h;
  return fmaf(fy, bot - top, top);
}

// The two Gauss points of [0, 1] (2-point rule), as compile-time constants.
constexpr float kGP0 = 0.21132486540518711775f, kGP1 = 0.78867513459481288225f;

// A bilinear field on one element (nodes 00, 10, 01, 11 as v[0..3]) at the 2x2 Gauss points:
// interpolated along x on the element's two rows, then along y.
struct QuadField {
  float top[2], dy[2];
  __device__ __forceinline__ explicit QuadField(const float (&v)[4]) {
    float d0 = v[1] - v[0], d1 = v[3] - v[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const float xi = q ? kGP1 : kGP0;
      top[q] = fmaf(xi, d0, v[0]);
      dy[q] = fmaf(xi, d1, v[2]) - top[q];
    }
  }
  __device__ __forceinline__ float at(int p, int q) const {
    return fmaf(p ? kGP1 : kGP0, dy[q], top[q]);
  }
};

// Clamped bilinear sample of a level's frame at (tx, ty) cells from the node whose record
// offset is base16 (bytes), for the energy passes, from the frame's coefficient records (C, a
// scalar base; n16 the row pitch in bytes). The position is clamped to the level ([lo, hi] are
// the level's bounds relative to that node); the cell is floor of the clamped position and the
// fraction its remainder, so a position on the far edge takes the last node at fraction 0 (its
// value, as with the cell before it at fraction 1). c0 + fx c1 + fy (c2 + fx c3).
__device__ __forceinline__ float sample_cells(const float* C, unsigned n16, unsigned base16,
                                              float lox, float hix, float loy, float hiy,
                                              float tx, float ty) {
  float cx = __builtin_amdgcn_fmed3f(tx, lox, hix);
  float cy = __builtin_amdgcn_fmed3f(ty, loy, hiy);
  int ix = cvt_flr(cx), iy = cvt_flr(cy);
  float fx = __builtin_amdgcn_fractf(cx), fy = __builtin_amdgcn_fractf(cy);
  unsigned o = (unsigned)mad24(iy, (int)n16, (int)(base16 + ((unsigned)ix << 4)));
  f32x4 c = ld_coef(C, o);
  return fmaf(fy, fmaf(fx, c.w, c.z), fmaf(fx, c.y, c.x));
}

// One DPP step of a wave reduction on a double: each lane the row mask enables takes the value
// of the lane the DPP control names, and 0 where that lane lies outside the row (or the lane
// is not enabled). Both halves move through the same lane pattern. All 64 lanes must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_take(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}
// A row shift of a double by DPP with bound control: a lane whose source lies outside its row
// reads 0 (every lane is written, so no zeroed destination is needed).
template <int CTRL>
__device__ __forceinline__ double dpp_shr(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, true);
  int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned)lo));
}
// DPP controls: row_shr:k (k = 1, 2, 4, 8), row_bcast:15 (lane 15 of a row into the next row),
// row_bcast:31 (lane 31 into rows 2 and 3)
enum { kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118,
       kRowBcast15 = 0x142, kRowBcast31 = 0x143 };

// Wave-level (64 lanes) sum of a double in a fixed order: running sums within each 16-lane
// row (lane 15 of a row then holds the row), then rows 0+1 and 2+3, then the two halves. The
// total is in lane 63 (kTotalLane).
const int kTotalLane = 63;
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_shr<kRowShr1>(v);
  v += dpp_shr<kRowShr2>(v);
  v += dpp_shr<kRowShr4>(v);
  v += dpp_shr<kRowShr8>(v);
  v += dpp_take<kRowBcast15, 0xa>(v);
  v += dpp_take<kRowBcast31, 0xc>(v);
  return v;
}
// The same pattern for the maximum of non-negative doubles (0 is the identity); lane 63.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_shr<kRowShr1>(v));
  v = fmax(v, dpp_shr<kRowShr2>(v));
  v = fmax(v, dpp_shr<kRowShr4>(v));
  v = fmax(v, dpp_shr<kRowShr8>(v));
  v = fmax(v, dpp_take<kRowBcast15, 0xa>(v));
  v = fmax(v, dpp_take<kRowBcast31, 0xc>(v));
  return v;
}

// Deterministic block reduction of NV doubles per thread (blockDim.x == BLOCK).
// Result valid in thread 0. scratch: BLOCK/64 * NV doubles.
template <int NV>
__device__ void block_sum(double (&v)[NV], double* scratch, bool is_max_last = false) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = (is_max_last && k == NV - 1) ? wave_max(v[k]) : wave_sum(v[k]);
    if (lane == kTotalLane) scratch[w * NV + k] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = scratch[k];
      for (int ww = 1; ww < BLOCK / 64; ++ww)
        s = (is_max_last && k == NV - 1) ? fmax(s, scratch[ww * NV + k]) : s + scratch[ww * NV + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Deterministic block reduction of NV doubles per thread (blockDim.x == BLOCK) with the totals
// stored to out[0..NV) in global memory. Per group of up to BLOCK / 16 values: one DPP step
// adds each odd lane's left neighbour, the BLOCK / 2 pair sums of each value go to LDS, and one
// 16-lane row per value adds its entries (lane j: entries j, j + 16, ..., in order), then the
// row's running sums leave the total in the row's last lane, which stores it. stage: at least
// min(NV, BLOCK / 16) * BLOCK / 2 doubles of LDS, free for this call's duration (it may alias
// the caller's tile buffers: the first barrier waits for every lane to be done with them).
// Far fewer instructions than a wave reduction per value.
template <int NV>
__device__ void block_sum_store(const double (&v)[NV], double* stage, double* out) {
  constexpr int KG = NV < BLOCK / 16 ? NV : BLOCK / 16, HALF = BLOCK / 2;
  const int tid = threadIdx.x, row = tid >> 4, sub = tid & 15;
#pragma unroll
  for (int k0 = 0; k0 < NV; k0 += KG) {
    __syncthreads();
#pragma unroll
    for (int k = k0; k < k0 + KG && k < NV; ++k) {
      double p = v[k] + dpp_shr<kRowShr1>(v[k]);
      if (tid & 1) stage[(k - k0) * HALF + (tid >> 1)] = p;
    }
    __syncthreads();
    if (row < KG && k0 + row < NV) {
      const double* src = stage + row * HALF + sub;
      double t = src[0];
#pragma unroll
      for (int j = 1; j < HALF / 16; ++j) t += src[16 * j];
      t += dpp_shr<kRowShr1>(t);
      t += dpp_shr<kRowShr2>(t);
      t += dpp_shr<kRowShr4>(t);
      t += dpp_shr<kRowShr8>(t);
      if (sub == 15) out[k0 + row] = t;
    }
  }
}

__device__ __forceinline__ float* slot_u(const BatchDesc* D, int s, int l, int buf) {
  int n = lvl_n(l);
  return D->ubuf + (size_t)s * D->slot_u_stride + D->u_off[l] + (size_t)buf * 2 * n * n;
}

// Copies of a slot's scalar fields (everything before the per-level arrays).
__device__ __forceinline__ void load_head(SlotState& dst, const SlotState& src) {
  dst.phase = src.phase; dst.level = src.level; dst.ub = src.ub; dst.iter = src.iter;
  dst.flags = src.flags; dst.ref = src.ref; dst.tmpl = src.tmpl; dst.finest = src.finest;
  dst.coarsest = src.coarsest; dst.rung = src.rung; dst.E = src.E; dst.ncc = src.ncc; dst.mean = src.mean;
  dst.sigma = src.sigma; dst.tau_prev = src.tau_prev; dst.top = src.top;
  dst.tau_max = src.tau_max; dst.tau_pend = src.tau_pend; dst.gtd = src.gtd; dst.dmax = src.dmax;
  for (int k = 0; k < 3; ++k) {
    dst.rp[k] = src.rp[k];
    dst.rd[k] = src.rd[k];
  }
}
__device__ __forceinline__ void store_head(SlotState& dst, const SlotState& src) {
  load_head(dst, src);
}

__device__ __forceinline__ void level_done(SlotState& st) {
  st.phase = st.level < st.finest ? PH_PROLONG : PH_DONE;
}

// Items of a kind for a slot whose effective level is l.
__device__ __forceinline__ int kind_items(const BatchDesc* D, int kind, int l) {
  const LevelGeom& g = D->geom[l];
  switch (kind) {
    case WK_PROLONG: return g.tiles_prol;
    case WK_EVAL: return g.tiles_elem;
    case WK_LADDER: return g.tiles_elem;
    case WK_GRAD: return g.tiles_grad;
    case WK_SMY: return D->smooth_halo ? 0 : 2 * g.sm_items;
    default: return D->smooth_halo ? 2 * g.sw_tiles * g.sw_tiles : 2 * g.sm_items;
  }
}

// ------------------------------------------------------------------------------------------
// Work distribution: workgroup b handles the contiguous item range
// [b * chunk, min((b+1) * chunk, total)); item -> (list position, local index).
// XGROUP > 0 (one item per workgroup only): workgroups go to the 8 XCDs in turn, each XCD with
// its own L2, so items are placed XGROUP consecutive ones to an XCD instead: workgroup
// b = 8 j + x takes item (j / XGROUP) 8 XGROUP + x XGROUP + j mod XGROUP, a permutation of
// [0, gridDim.x) when gridDim.x is a multiple of 8 XGROUP. Neighbouring items that read two
// halves of the same 128-byte lines then fetch them into one L2.

struct ItemCursor {
  int item, end, pos;
};

template <int XGROUP>
__device__ __forceinline__ int placed_block(int chunk) {
  int b = blockIdx.x;
  if (XGROUP > 0 && chunk == 1 && gridDim.x % (8 * XGROUP) == 0) {
    int x = b & 7, j = b >> 3;
    b = (j / XGROUP) * (8 * XGROUP) + x * XGROUP + j % XGROUP;
  }
  return b;
}

template <int XGROUP = 0>
__device__ bool cursor_begin(const BatchDesc* D, int kind, ItemCursor& c, int* s_pos) {
  const WorkList wl = D->lists[kind];
  int total = wl.total;
  if (total <= 0) return false;
  int chunk = (total + gridDim.x - 1) / gridDim.x;
  c.item = placed_block<XGROUP>(chunk) * chunk;
  c.end = min(c.item + chunk, total);
  if (c.item >= c.end) return false;
  if (threadIdx.x == 0) {
    const int* off = D->list_off + (size_t)kind * (D->max_slots + 1);
    int lo = 0, hi = wl.n_slots - 1;
    while (lo < hi) {  // largest pos with off[pos] <= item
      int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= c.item) lo = mid; else hi = mid - 1;
    }
    *s_pos = lo;
  }
  __syncthreads();
  c.pos = __builtin_amdgcn_readfirstlane(*s_pos);  // block-uniform
  __syncthreads();
  return true;
}

// The items [item0, item1) of one list (uniform over the block; false when empty).
__device__ bool cursor_range(const BatchDesc* D, int kind, int item0, int item1, ItemCursor& c,
                             int* s_pos) {
  if (item0 >= item1) return false;
  c.item = item0;
  c.end = item1;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int* off = D->list_off + (size_t)kind * (D->max_slots + 1);
    int lo = 0, hi = D->lists[kind].n_slots - 1;
    while (lo < hi) {  // largest pos with off[pos] <= item
      int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= c.item) lo = mid; else hi = mid - 1;
    }
    *s_pos = lo;
  }
  __syncthreads();
  c.pos = __builtin_amdgcn_readfirstlane(*s_pos);  // block-uniform
  __syncthreads();
  return true;
}

__device__ __forceinline__ void cursor_slot(const BatchDesc* D, int kind, ItemCursor& c,
                                            int& slot, int& local) {
  const int* off = D->list_off + (size_t)kind * (D->max_slots + 1);
  while (c.item >= off[c.pos + 1]) c.pos++;
  slot = D->list_slots[(size_t)kind * D->max_slots + c.pos];
  local = c.item - off[c.pos];
}

__device__ __forceinline__ double* slot_partial(const BatchDesc* D, int s, int kind, int item) {
  return D->partial + (size_t)s * D->part_slot_stride + (size_t)kind * D->part_kind_stride +
         (size_t)item * PW;
}

// Fixed-order sum of NV columns over n_items partial records; result in thread 0's out[].
// (Compile-time NV keeps out[] in registers; a record's NV loads are issued together.)
// partials_local: each thread's share (records threadIdx.x, + BLOCK, ...); sum_partials: that
// and the block reduction.
template <int NV>
__device__ __forceinline__ void partials_local(const BatchDesc* D, int s, int kind, int n_items,
                                               double (&out)[NV], bool max_last) {
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = 0.0;
  for (int it = threadIdx.x; it < n_items; it += BLOCK) {
    const double* p = slot_partial(D, s, kind, it);
    double x[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) x[k] = p[k];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      if (max_last && k == NV - 1) out[k] = fmax(out[k], x[k]);
      else out[k] += x[k];
    }
  }
}
template <int NV>
__device__ __forceinline__ void sum_partials(const BatchDesc* D, int s, int kind, int n_items,
                                             double (&out)[NV], double* scratch, bool max_last) {
  partials_local<NV>(D, s, kind, n_items, out, max_last);
  block_sum<NV>(out, scratch, max_last);
}

// ------------------------------------------------------------------------------------------
// Planning kernel: one workgroup of PLAN_T threads, a slot per thread and round.

#define PLAN_T 512
#define PLAN_V (2 * WK_COUNT)
template <int NT>
struct PlanLds {
  int wtot[NT / 64][PLAN_V];
  int woff[NT / 64][PLAN_V];
  int carry[PLAN_V];
  int active[NT / 64];
  int items[PPRS_MAXL][WK_COUNT];  // kind_items per effective level
};

// Inclusive scan of an int over the 64 lanes of a wave on DPP moves: running sums inside each
// 16-lane row, then row 0 into row 1 and row 2 into row 3 (row_bcast:15), then rows 0-1 into
// rows 2-3 (row_bcast:31). A lane reading outside its row, or not enabled, adds 0.
__device__ __forceinline__ int wave_scan_incl(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, kRowShr1, 0xf, 0xf, true);
  v += __builtin_amdgcn_update_dpp(0, v, kRowShr2, 0xf, 0xf, true);
  v += __builtin_amdgcn_update_dpp(0, v, kRowShr4, 0xf, 0xf, true);
  v += __builtin_amdgcn_update_dpp(0, v, kRowShr8, 0xf, 0xf, true);
  v += __builtin_amdgcn_update_dpp(0, v, kRowBcast15, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, kRowBcast31, 0xc, 0xf, false);
  return v;
}

// One workgroup of NT threads: per kind, the compacted list of member slots and the prefix sum
// of their item counts. The item counts per level come from a table in LDS (filled while the
// slot states load); wave-level DPP scans, then a scan over the wave totals.
template <int NT>
__device__ void plan_body(BatchDesc* D, PlanLds<NT>& P) {
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int n_slots = D->n_slots;
  int active = 0;
  if (threadIdx.x < PLAN_V) P.carry[threadIdx.x] = 0;
  if (threadIdx.x < PPRS_MAXL * WK_COUNT) {
    int l = threadIdx.x / WK_COUNT, k = threadIdx.x - l * WK_COUNT;
    P.items[l][k] = (l >= D->coarsest && l <= D->finest) ? kind_items(D, k, l) : 0;
  }
  for (int base = 0; base < n_slots; base += NT) {
    int s = base + threadIdx.x;
    int ph = PH_DONE, eff = 0;
    if (s < n_slots) {
      const SlotState* st = D->state + s;
      ph = st->phase;
      eff = ph == PH_PROLONG ? st->level + 1 : st->level;
    }
    __syncthreads();  // the table and the carries (and the previous round's offsets)
    active += ph != PH_DONE;
    int val[PLAN_V];
#pragma unroll
    for (int k = 0; k < WK_COUNT; ++k) {
      bool m;
      // A slot that begins a level this step (INIT, PROLONG) takes its start energy only, at
      // the end of the step beside the line searches; its first iteration is the next step's.
      // The iterating slots (GRAD, LADDER) take gradient, metric solve and line search.
      switch (k) {
        case WK_PROLONG: m = ph == PH_PROLONG; break;
        case WK_EVAL: m = ph == PH_PROLONG || ph == PH_INIT; break;
        case WK_LADDER: m = ph == PH_GRAD || ph == PH_LADDER; break;
        default: m = ph == PH_GRAD; break;
      }
      val[2 * k] = m ? 1 : 0;
      val[2 * k + 1] = m ? P.items[eff][k] : 0;
    }
    int inc[PLAN_V];
#pragma unroll
    for (int v = 0; v < PLAN_V; ++v) inc[v] = wave_scan_incl(val[v]);
    if (lane == 63)
#pragma unroll
      for (int v = 0; v < PLAN_V; ++v) P.wtot[wv][v] = inc[v];
    __syncthreads();
    if (threadIdx.x < PLAN_V) {
      int v = threadIdx.x, acc = P.carry[v];
      for (int w = 0; w < NT / 64; ++w) {
        P.woff[w][v] = acc;
        acc += P.wtot[w][v];
      }
      P.carry[v] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < WK_COUNT; ++k) {
      if (val[2 * k]) {
        int pos = P.woff[wv][2 * k] + inc[2 * k] - 1;
        int off = P.woff[wv][2 * k + 1] + inc[2 * k + 1] - val[2 * k + 1];
        D->list_slots[(size_t)k * D->max_slots + pos] = s;
        D->list_off[(size_t)k * (D->max_slots + 1) + pos] = off;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) active += __shfl_down(active, o, 64);
  if (lane == 0) P.active[wv] = active;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int w = 0; w < NT / 64; ++w) tot += P.active[w];
    D->active = tot;
  }
  if (threadIdx.x < WK_COUNT) {
    int k = threadIdx.x;
    int cnt = P.carry[2 * k], items = P.carry[2 * k + 1];
    D->list_off[(size_t)k * (D->max_slots + 1) + cnt] = items;
    D->lists[k].n_slots = cnt;
    D->lists[k].total = items;
  }
}

__global__ void __launch_bounds__(PLAN_T) k_plan(BatchDesc* D) {
  __shared__ PlanLds<PLAN_T> P;
  plan_body<PLAN_T>(D, P);
}

// ------------------------------------------------------------------------------------------
// Prolongation of u (level l -> l+1) with the pending step applied: u_l - tau_pend d.

// One prolongation item: fine-level tile t of slot s.
__device__ __forceinline__ void prolong_item(BatchDesc* D, int s, int t) {
  {
    const SlotState& st = D->state[s];
    if (st.phase != PH_PROLONG) return;
    int lc = st.level, lf = lc + 1;
    int nc = lvl_n(lc), nf = lvl_n(lf);
    const float* uc = slot_u(D, s, lc, st.ub);
    const float* dd = D->dbuf + (size_t)s * D->slot_f_stride;
    float tau = (float)st.tau_pend;
    float* uf = slot_u(D, s, lf, 0);
    int ntx = (nf + PT_X - 1) / PT_X;
    int x0 = (t % ntx) * PT_X, y0 = (t / ntx) * PT_Y;
    size_t ncc = (size_t)nc * nc, nff = (size_t)nf * nf;
    for (int k = threadIdx.x; k < PT_X * PT_Y; k += BLOCK) {
      int a = y0 + k / PT_X, b = x0 + k % PT_X;
      if (a >= nf || b >= nf) continue;
      int A = a >> 1, B = b >> 1;
      int A1 = (a & 1) ? A + 1 : A, B1 = (b & 1) ? B + 1 : B;
      for (int comp = 0; comp < 2; ++comp) {
        const float* u = uc + comp * ncc;
        const float* d = dd + comp * ncc;
        size_t i00 = (size_t)A * nc + B, i01 = (size_t)A * nc + B1;
        size_t i10 = (size_t)A1 * nc + B, i11 = (size_t)A1 * nc + B1;
        float v00 = u[i00], v01 = u[i01], v10 = u[i10], v11 = u[i11];
        if (tau != 0.f) {
          v00 -= tau * d[i00];
          v01 -= tau * d[i01];
          v10 -= tau * d[i10];
          v11 -= tau * d[i11];
        }
        uf[comp * nff + (size_t)a * nf + b] = 0.25f * ((v00 + v01) + (v10 + v11));
      }
    }
  }
}


// Element stiffness (Q1, h-independent in 2-D), corners ordered 00, 01, 10, 11: diagonal 2/3,
// edge pairs -1/6, opposite pairs -1/3. Its rows sum to zero, so the bilinear form is written
// with node differences, which keeps FP32 free of cancellation for nearly constant fields:
//   a^T K_e b = 1/6 sum_edges (a_i - a_j)(b_i - b_j) + 1/3 sum_opposite (a_i - a_j)(b_i - b_j).
__device__ __forceinline__ float ke_form(float a0, float a1, float a2, float a3, float b0,
                                         float b1, float b2, float b3) {
  float edge = (a0 - a1) * (b0 - b1) + (a0 - a2) * (b0 - b2) + (a1 - a3) * (b1 - b3) +
               (a2 - a3) * (b2 - b3);
  float opp = (a0 - a3) * (b0 - b3) + (a1 - a2) * (b1 - b2);
  return (1.f / 6.f) * edge + (1.f / 3.f) * opp;
}

// (K_e u)_k = 1/6 sum over edge neighbours j of (u_k - u_j) + 1/3 (u_k - u_opposite).
__device__ __forceinline__ void ke_apply(const float u[4], float out[4]) {
  float d01 = u[0] - u[1], d02 = u[0] - u[2], d13 = u[1] - u[3], d23 = u[2] - u[3];
  float d03 = u[0] - u[3], d12 = u[1] - u[2];
  out[0] = (1.f / 6.f) * (d01 + d02) + (1.f / 3.f) * d03;
  out[1] = (1.f / 6.f) * (d13 - d01) + (1.f / 3.f) * d12;
  out[2] = (1.f / 6.f) * (d23 - d02) - (1.f / 3.f) * d12;
  out[3] = (1.f / 6.f) * (-d13 - d23) - (1.f / 3.f) * d03;
}

// ------------------------------------------------------------------------------------------
// Energy kernel. MODE 0: energy of the starting u of a level (slots in INIT or PROLONG).
// MODE 1: one line-search pass at NC = 2K+1 step sizes (slots in LADDER).
// Per element tile: quadrature sums S1 = sum w T, S2 = sum w T^2, S3 = sum w R~ T for each
// step size, and the Dirichlet terms u^T K u, d^T K u, d^T K d via element matrices.

// The finaliser's operands in global memory outside the slot's head: the reference's
// quadrature sum on the level, the slot's node counters, its probe flag and the pass count of
// its level, and the run's parameters. Thread 0 loads them before the block reduction, so that
// their latency overlaps it instead of following it load after load (a read after the first
// store would otherwise wait for it); only the slot's own finaliser writes them within a launch.
struct FinOperands {
  double rsum;
  long long nodes_kind, nodes_prol;
  int eval_only, passes;
  double sigma, tau_min_rel, eps;
  int iter_max, rigid;
  unsigned char* dlog;
};
template <int MODE>
__device__ __forceinline__ void load_fin_operands(const BatchDesc* D, const SlotState* stp,
                                                  const SlotState& st, int s, int l,
                                                  FinOperands& fo) {
  const int kind = MODE ? WK_LADDER : WK_EVAL;
  const long long* nc_s = D->node_count + (size_t)s * WK_COUNT;
  fo.rsum = D->rsum[(size_t)st.ref * PPRS_MAXL + l];
  fo.nodes_kind = nc_s[kind];
  fo.nodes_prol = MODE ? 0 : nc_s[WK_PROLONG];
  fo.eval_only = MODE ? 0 : stp->eval_only;
  fo.passes = MODE ? stp->passes[st.level - st.coarsest] : 0;
  fo.sigma = D->sigma;
  fo.tau_min_rel = D->tau_min_rel;
  fo.eps = D->eps;
  fo.iter_max = D->iter_max;
  fo.rigid = D->rigid;
  fo.dlog = D->dlog;
}

// Works on a register copy of the slot's scalar fields (loaded together up front, stored back
// at the end): every read of global state would otherwise wait behind the previous store.
template <int MODE, int NC>
__device__ __forceinline__ void energy_finalize(BatchDesc* D, SlotState* stp, SlotState& st,
                                                int s, int l, int n, int ph, double top,
                                                const double (&tot)[3 * NC + 3],
                                                const FinOperands& fo) {
  const int kind = MODE ? WK_LADDER : WK_EVAL;
  int K = D->ladder_k;
  double rs = fo.rsum;
  double e_j[NC], ncc_j[NC], m_j[NC], sg_j[NC];
  for (int j = 0; j < NC; ++j) {
    double m = tot[3 * j], var = tot[3 * j + 1] - m * m;
    double sg = var > 0.0 ? sqrt(var) : 0.0;
    double ncc = sg > 0.0 ? (tot[3 * j + 2] - m * rs) / sg : 0.0;
    double tj = MODE ? ldexp(top, -j) : 0.0;
    double reg = tot[3 * NC] - 2.0 * tj * tot[3 * NC + 1] + tj * tj * tot[3 * NC + 2];
    e_j[j] = -ncc + 0.5 * D->lambda * reg;
    ncc_j[j] = ncc;
    m_j[j] = m;
    sg_j[j] = sg;
  }
  long long* nc_s = D->node_count + (size_t)s * WK_COUNT;
  nc_s[kind] = fo.nodes_kind + (long long)n * n;
  if (MODE == 0 && ph == PH_PROLONG) nc_s[WK_PROLONG] = fo.nodes_prol + (long long)n * n;
  if (MODE == 0) {
    if (ph == PH_PROLONG) {
      st.level = l;
      st.ub = 0;
    }
    st.iter = 0;
    st.tau_prev = INFINITY;
    st.tau_pend = 0.0;
    st.E = e_j[0];
    st.ncc = ncc_j[0];
    st.mean = m_j[0];
    st.sigma = sg_j[0];
    if (!isfinite(st.E)) {
      st.flags |= FLAG_NAN;
      st.phase = PH_DONE;
    } else if (fo.iter_max <= 0 || fo.eval_only) {
      level_done(st);
    } else {
      st.phase = PH_GRAD;
    }
  } else {
    // The pass evaluated NC consecutive steps of the ladder tau = top 2^-j; the ladder is taken
    // in groups of G = 2K+1 steps, and a group whose first step is below tau_min_rel * tau_max
    // is not started. Walking the steps in order with that rule gives the same accepted step
    // and group count for any NC (NC is a launch-shape choice).
    const int G = 2 * K + 1;
    const double tmin = fo.tau_min_rel * st.tau_max;
    int li = st.level - st.coarsest;
    int r = st.rung;
    int acc_j = -1;
    bool stop = false;
    int passes = fo.passes;
    for (int j = 0; j < NC; ++j, ++r) {
      double tj = ldexp(top, -j);
      if (r == G) {
        r = 0;
        if (tj < tmin) {
          stop = true;
          break;
        }
      }
      if (r == 0) passes++;
      if (e_j[j] <= st.E - fo.sigma * tj * st.gtd) {
        acc_j = j;
        break;
      }
    }
    if (passes != fo.passes) stp->passes[li] = passes;
    if (acc_j >= 0) {
      double tj = ldexp(top, -acc_j);
      double dec = st.E - e_j[acc_j];
      if (fo.dlog) {
        // ladder position of the accepted step: tj = top0 2^-J, top0 the iteration's first
        // step (powers of two apart, so the exponents differ by exactly J)
        int pos = st.iter;
        for (int k = 0; k < li; ++k) pos += stp->iters[k];
        if (pos < D->dlog_cap) {
          double top0 = fmin(ldexp(st.tau_prev, K), st.tau_max);
          int J = ilogb(top0) - ilogb(tj);
          D->dlog[(size_t)stp->op * D->dlog_cap + pos] = (unsigned char)min(max(J, 0), 255);
        }
      }
      st.E = e_j[acc_j];
      st.ncc = ncc_j[acc_j];
      st.mean = m_j[acc_j];
      st.sigma = sg_j[acc_j];
      if (fo.rigid) {
        for (int k = 0; k < 3; ++k) st.rp[k] -= tj * st.rd[k];  // parameters move at once
      } else {
        st.tau_pend = tj;  // applied to u by the next gradient pass
      }
      st.tau_prev = tj;
      st.iter++;
      stp->iters[li] = st.iter;
      if (dec < fo.eps) {
        level_done(st);
      } else if (st.iter >= fo.iter_max) {
        st.flags |= FLAG_NONCONV;
        level_done(st);
      } else {
        st.phase = PH_GRAD;
      }
    } else if (stop) {
      level_done(st);
    } else {
      // next pass: the step after the last one evaluated
      st.top = ldexp(top, -NC);
      if (r == G) {
        r = 0;
        if (st.top < tmin) stop = true;
      }
      st.rung = r;
      if (stop) level_done(st);
      else st.phase = PH_LADDER;
    }
  }
  store_head(*stp, st);
}

// Staged nodes of an element tile (ET_X x ET_Y elements).
#define ET_NN ((ET_X + 1) * (ET_Y + 1))

// One energy item: element tile t of slot s (MODE 0: the start energy of a level; MODE 1: a
// line-search pass at NC step sizes). The LDS arrays are the caller's (s_dx, s_dy unused in
// MODE 0).
template <int MODE, int NC>
__device__ __forceinline__ void energy_item(BatchDesc* D, int s, int t, float* s_ux, float* s_uy,
                                            float* s_dx, float* s_dy, float* s_r,
                                            double* s_stage) {
  constexpr int NXN = ET_X + 1, NN = ET_NN;
  constexpr int NV = 3 * NC + 3;
  const int kind = MODE ? WK_LADDER : WK_EVAL;
  {
    SlotState* stp = D->state + s;
    int ph = stp->phase;
    if (MODE == 0 && !(ph == PH_INIT || ph == PH_PROLONG)) return;
    if (MODE == 1 && ph != PH_LADDER) return;
    int l = (ph == PH_PROLONG) ? stp->level + 1 : stp->level;
    int ub = (ph == PH_PROLONG) ? 0 : stp->ub;
    int n = lvl_n(l);
    size_t nn = (size_t)n * n;
    const float* u = uni(slot_u(D, s, l, ub));
    const float* d = uni(D->dbuf + (size_t)s * D->slot_f_stride);
    const float* R = uni(D->pyr + D->frame_off[(size_t)stp->ref * PPRS_MAXL + l]);
    const float* TC = uni(D->tcoef + 4 * D->frame_off[(size_t)stp->tmpl * PPRS_MAXL + l]);
    const unsigned nn4 = (unsigned)nn << 2;
    double top = MODE ? stp->top : 0.0;
    float taus[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) taus[j] = MODE ? (float)ldexp(top, -j) : 0.f;
    float inv_h = (float)(n - 1);
    int ntx = (n - 1 + ET_X - 1) / ET_X;
    int e0x = (t % ntx) * ET_X, e0y = (t / ntx) * ET_Y;
    // stage the nodes of the tile's elements: every load of a lane is issued before the first
    // LDS store (out-of-range nodes load node 0 and store zero), so a lane waits for memory
    // once per item instead of once per strided round
    __syncthreads();
    {
      constexpr int SIT = (NN + BLOCK - 1) / BLOCK;
      float vux[SIT], vuy[SIT], vr[SIT], vdx[SIT], vdy[SIT];
#pragma unroll
      for (int it = 0; it < SIT; ++it) {
        int k = threadIdx.x + it * BLOCK;
        int a = e0y + k / NXN, b = e0x + k % NXN;
        unsigned o = ((k < NN) & (a < n) & (b < n)) ? (unsigned)mad24(a, n, b) << 2 : 0u;
        vux[it] = ldo(u, o);
        vuy[it] = ldo(u, nn4 + o);
        vr[it] = ldo(R, o);
        if (MODE) {
          vdx[it] = ldo(d, o);
          vdy[it] = ldo(d, nn4 + o);
        }
      }
#pragma unroll
      for (int it = 0; it < SIT; ++it) {
        int k = threadIdx.x + it * BLOCK;
        int a = e0y + k / NXN, b = e0x + k % NXN;
        if (k >= NN) break;
        bool ok = a < n && b < n;
        // displacements in cells of the level (a power-of-two scaling: exact)
        s_ux[k] = ok ? vux[it] * inv_h : 0.f;
        s_uy[k] = ok ? vuy[it] * inv_h : 0.f;
        s_r[k] = ok ? vr[it] : 0.f;
        if (MODE) {
          s_dx[k] = ok ? vdx[it] * inv_h : 0.f;
          s_dy[k] = ok ? vdy[it] * inv_h : 0.f;
        }
      }
    }
    __syncthreads();
    // per-thread FP32 sums over the thread's elements of the tile (at most
    // ET_X * ET_Y / BLOCK), converted to FP64 once per tile
    float es[3 * NC], dir[3];
#pragma unroll
    for (int k = 0; k < 3 * NC; ++k) es[k] = 0.f;
    dir[0] = dir[1] = dir[2] = 0.f;
    const unsigned n16 = (unsigned)n << 4;
    for (int e = threadIdx.x; e < ET_X * ET_Y; e += BLOCK) {
      int ey = e / ET_X, ex = e % ET_X;
      int a = e0y + ey, b = e0x + ex;
      if (a >= n - 1 || b >= n - 1) continue;
      int k00 = ey * NXN + ex;
      float ux[4] = {s_ux[k00], s_ux[k00 + 1], s_ux[k00 + NXN], s_ux[k00 + NXN + 1]};
      float uy[4] = {s_uy[k00], s_uy[k00 + 1], s_uy[k00 + NXN], s_uy[k00 + NXN + 1]};
      float rr[4] = {s_r[k00], s_r[k00 + 1], s_r[k00 + NXN], s_r[k00 + NXN + 1]};
      float dx[4] = {0, 0, 0, 0}, dy[4] = {0, 0, 0, 0};
      if (MODE) {
        dx[0] = s_dx[k00]; dx[1] = s_dx[k00 + 1]; dx[2] = s_dx[k00 + NXN]; dx[3] = s_dx[k00 + NXN + 1];
        dy[0] = s_dy[k00]; dy[1] = s_dy[k00 + 1]; dy[2] = s_dy[k00 + NXN]; dy[3] = s_dy[k00 + NXN + 1];
      }
      // Dirichlet terms (in cells: h^2 times the domain-unit forms)
      dir[0] += ke_form(ux[0], ux[1], ux[2], ux[3], ux[0], ux[1], ux[2], ux[3]) +
                ke_form(uy[0], uy[1], uy[2], uy[3], uy[0], uy[1], uy[2], uy[3]);
      if (MODE) {
        dir[1] += ke_form(dx[0], dx[1], dx[2], dx[3], ux[0], ux[1], ux[2], ux[3]) +
                  ke_form(dy[0], dy[1], dy[2], dy[3], uy[0], uy[1], uy[2], uy[3]);
        dir[2] += ke_form(dx[0], dx[1], dx[2], dx[3], dx[0], dx[1], dx[2], dx[3]) +
                  ke_form(dy[0], dy[1], dy[2], dy[3], dy[0], dy[1], dy[2], dy[3]);
      }
      // the element's cell in the clamp bounds and the byte offset of its first node
      const float lox = (float)(-b), hix = (float)(n - 1 - b);
      const float loy = (float)(-a), hiy = (float)(n - 1 - a);
      const unsigned base16 = (unsigned)mad24(a, n, b) << 4;
      // 2x2 Gauss points, fields interpolated along x first (rows of the element), then y
      QuadField qux(ux), quy(uy), qr(rr), qdx(dx), qdy(dy);
#pragma unroll
      for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float xi = q ? kGP1 : kGP0, eta = p ? kGP1 : kGP0;
          // the Gauss point's position in cells from the element's first node, at tau = 0
          float px = qux.at(p, q) + xi, py = quy.at(p, q) + eta, rq = qr.at(p, q);
          float dqx = MODE ? qdx.at(p, q) : 0.f, dqy = MODE ? qdy.at(p, q) : 0.f;
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            float tx = fmaf(-taus[j], dqx, px);
            float ty = fmaf(-taus[j], dqy, py);
            float tv = sample_cells(TC, n16, base16, lox, hix, loy, hiy, tx, ty);
            es[3 * j + 0] += tv;
            es[3 * j + 1] = fmaf(tv, tv, es[3 * j + 1]);
            es[3 * j + 2] = fmaf(tv, rq, es[3 * j + 2]);
          }
        }
      }
    }
    double acc[NV];
    const double w = 0.25 / ((double)(n - 1) * (double)(n - 1));
    const double h2 = 1.0 / ((double)(n - 1) * (double)(n - 1));
#pragma unroll
    for (int k = 0; k < 3 * NC; ++k) acc[k] = w * (double)es[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[3 * NC + k] = h2 * (double)dir[k];
    // s_stage aliases the tile buffers
    block_sum_store<NV>(acc, s_stage, slot_partial(D, s, kind, t));
  }
}

// LDS of an energy workgroup: the tile's staged fields (NF arrays of ET_NN floats), also the
// stage of the partial-sum reduction once the tile is done.
template <int NF, int NV>
struct EnergyLds {
  static constexpr int FLOATS = NF * ET_NN, KG = NV < BLOCK / 16 ? NV : BLOCK / 16;
  static_assert(FLOATS / 2 >= KG * (BLOCK / 2), "reduction stage fits the tile buffers");
  double buf[(FLOATS + 1) / 2];
  __device__ float* field(int i) { return reinterpret_cast<float*>(buf) + i * ET_NN; }
};

// The energy passes of a step in one launch: the start energies of the slots that begin a
// level (the eval list) and the line-search passes (the ladder list), one item space made of
// the two lists in that order. The two slot sets are disjoint (the plan gives a slot that
// begins a level no gradient work in the same step).
template <int NC>
__global__ void __launch_bounds__(BLOCK, LB_ENERGY) k_energy_step(BatchDesc* D) {
  __shared__ EnergyLds<5, 3 * NC + 3> L;
  float *s_ux = L.field(0), *s_uy = L.field(1), *s_r = L.field(2), *s_dx = L.field(3),
        *s_dy = L.field(4);
  __shared__ int s_pos;
  const int ne = D->lists[WK_EVAL].total, nl = D->lists[WK_LADDER].total;
  const int total = ne + nl;
  if (total <= 0) return;
  int chunk = (total + gridDim.x - 1) / gridDim.x;
  int b0 = placed_block<16>(chunk) * chunk, b1 = min(b0 + chunk, total);
  ItemCursor c;
  if (b0 < ne && cursor_range(D, WK_EVAL, b0, min(b1, ne), c, &s_pos)) {
    for (; c.item < c.end; ++c.item) {
      int s, t;
      cursor_slot(D, WK_EVAL, c, s, t);
      energy_item<0, 1>(D, s, t, s_ux, s_uy, s_dx, s_dy, s_r, L.buf);
    }
  }
  if (b1 > ne && cursor_range(D, WK_LADDER, max(b0, ne) - ne, b1 - ne, c, &s_pos)) {
    for (; c.item < c.end; ++c.item) {
      int s, t;
      cursor_slot(D, WK_LADDER, c, s, t);
      energy_item<1, NC>(D, s, t, s_ux, s_uy, s_dx, s_dy, s_r, L.buf);
    }
  }
}

// Per-slot finalisation of an energy pass: one workgroup per listed slot sums the tile
// partials in tile order and advances the slot (the kernel boundary orders it after the pass).
// The slot's item count comes from the list offsets the plan wrote (the slot's tiles on the
// level it was listed for), so the partial loads do not wait for the slot state; a slot the
// metric-solve finaliser already moved off its line search is skipped after the sums.
template <int MODE, int NC>
__device__ __forceinline__ void energy_fin_slot(BatchDesc* D, int pos, double* s_red) {
  constexpr int NV = 3 * NC + 3;
  const int kind = MODE ? WK_LADDER : WK_EVAL;
  const int* off = D->list_off + (size_t)kind * (D->max_slots + 1);
  const int s = D->list_slots[(size_t)kind * D->max_slots + pos];
  const int n_items = off[pos + 1] - off[pos];
  SlotState* stp = D->state + s;
  SlotState st;
  load_head(st, *stp);  // in flight with the partial loads
  double tot[NV];
  partials_local<NV>(D, s, kind, n_items, tot, false);
  const int ph = st.phase;
  bool live = MODE == 0 ? (ph == PH_INIT || ph == PH_PROLONG) : ph == PH_LADDER;
  const int l = (ph == PH_PROLONG) ? st.level + 1 : st.level;
  FinOperands fo;
  if (live && threadIdx.x == 0) load_fin_operands<MODE>(D, stp, st, s, l, fo);
  block_sum<NV>(tot, s_red, false);
  if (live && threadIdx.x == 0)
    energy_finalize<MODE, NC>(D, stp, st, s, l, lvl_n(l), ph, MODE ? st.top : 0.0, tot, fo);
  __syncthreads();
}

// Finalisers of k_energy_step: the eval list's slots, then the ladder list's.
template <int NC>
__global__ void __launch_bounds__(BLOCK) k_energy_step_fin(BatchDesc* D) {
  constexpr int NV = 3 * NC + 3;
  __shared__ double s_red[(BLOCK / 64) * NV];
  const int ne = D->lists[WK_EVAL].n_slots, nl = D->lists[WK_LADDER].n_slots;
  for (int pos = blockIdx.x; pos < ne + nl; pos += gridDim.x) {
    if (pos < ne)
      energy_fin_slot<0, 1>(D, pos, s_red);
    else
      energy_fin_slot<1, NC>(D, pos - ne, s_red);
  }
}

// ------------------------------------------------------------------------------------------
// Gradient kernel (slots in GRAD): u_new = u - tau_pend d, written to the other u buffer;
// G_i = sum over the elements around node i of
//       sum_q psi_i(q) f_q grad T(q + u(q)) + lambda (K_e u_e)_i,
//       f_q = -w (R~(q) - NCC (T(q) - mean) / sigma) / sigma.

// Tile shape TX x TY nodes (a launch-shape choice: every node's G is the same sum of the same
// element terms whatever the tile, so the shape never changes a result). A level has 2^l + 1
// nodes per axis: the last tile of each row and column of tiles takes the extra node (TX + 1
// wide), so no tile is a one-node sliver.
template <int TX, int TY>
struct GradLds {
  static constexpr int NX = TX + 3, NY = TY + 3;  // staged nodes of the widest tile
  static constexpr int EX = TX + 2, EY = TY + 2;  // elements touching the widest tile
  float ux[NX * NY], uy[NX * NY], r[NX * NY];
  float c[8][EX * EY];                             // per element, per corner, (x, y)
};

// One gradient item: node tile t of slot s (the LDS block is the caller's).
template <int TX, int TY>
__device__ __forceinline__ void grad_item(BatchDesc* D, int s, int t, GradLds<TX, TY>& L) {
  constexpr int GT_X = TX, GT_Y = TY;
  static_assert((TX & (TX - 1)) == 0 && (TY & (TY - 1)) == 0, "tile sides are powers of two");
  constexpr int NX = GradLds<TX, TY>::NX, NY = GradLds<TX, TY>::NY;
  constexpr int EX = GradLds<TX, TY>::EX, EY = GradLds<TX, TY>::EY;
  float* s_ux = L.ux;
  float* s_uy = L.uy;
  float* s_r = L.r;
  auto& s_c = L.c;
  {
    const SlotState* stp = D->state + s;
    if (stp->phase != PH_GRAD) return;
    int l = stp->level;
    int n = lvl_n(l);
    size_t nn = (size_t)n * n;
    const float* u = uni(slot_u(D, s, l, stp->ub));
    float* un = uni(slot_u(D, s, l, stp->ub ^ 1));
    const float* d = uni(D->dbuf + (size_t)s * D->slot_f_stride);
    float* G = uni(D->gbuf + (size_t)s * D->slot_p_stride);
    const int gpi = row_pitch(n);
    const unsigned nn4 = (unsigned)nn << 2, gpn4 = (unsigned)(n * gpi) << 2;
    const float* R = uni(D->pyr + D->frame_off[(size_t)stp->ref * PPRS_MAXL + l]);
    const float* T = uni(D->pyr + D->frame_off[(size_t)stp->tmpl * PPRS_MAXL + l]);
    const float* T1 = uni(T + n);  // the row below, as a second scalar base
    const unsigned n4 = (unsigned)n << 2;
    float tau = (float)stp->tau_pend;
    double sg = stp->sigma;
    float inv_sig = sg > 0.0 ? (float)(1.0 / sg) : 0.f;
    float ncc = (float)stp->ncc, mean = (float)stp->mean;
    float lam = (float)D->lambda;
    float inv_h = (float)(n - 1);
    float w = 0.25f / ((float)(n - 1) * (float)(n - 1));
    const int ntx = max(1, (n - 1) / GT_X), nty = max(1, (n - 1) / GT_Y);
    const int txi = t % ntx, tyi = t / ntx;
    const int x0 = txi * GT_X, y0 = tyi * GT_Y;
    const int tw = txi == ntx - 1 ? n - x0 : GT_X;  // nodes of this tile (<= GT_X + 1)
    const int th = tyi == nty - 1 ? n - y0 : GT_Y;
    // stage u - tau d and R with the halo: all loads of a lane first, then the LDS stores
    __syncthreads();
    {
      constexpr int SIT = (NX * NY + BLOCK - 1) / BLOCK;
      float vux[SIT], vuy[SIT], vr[SIT], vdx[SIT], vdy[SIT];
      const bool mv = tau != 0.f;
      bool okv[SIT];
#pragma unroll
      for (int it = 0; it < SIT; ++it) {
        int k = threadIdx.x + it * BLOCK;
        int ky = k / NX, kx = k % NX;
        int a = y0 - 1 + ky, b = x0 - 1 + kx;
        okv[it] = (k < NX * NY) & (ky < th + 2) & (kx < tw + 2) & ((unsigned)a < (unsigned)n) &
                  ((unsigned)b < (unsigned)n);
        unsigned o = okv[it] ? (unsigned)mad24(a, n, b) << 2 : 0u;
        vux[it] = ldo(u, o);
        vuy[it] = ldo(u, nn4 + o);
        vr[it] = ldo(R, o);
        vdx[it] = mv ? ldo(d, o) : 0.f;
        vdy[it] = mv ? ldo(d, nn4 + o) : 0.f;
      }
#pragma unroll
      for (int it = 0; it < SIT; ++it) {
        int k = threadIdx.x + it * BLOCK;
        if (k >= NX * NY) break;
        float ux = 0.f, uy = 0.f, r = 0.f;
        if (okv[it]) {
          ux = vux[it];
          uy = vuy[it];
          if (mv) {
            ux -= tau * vdx[it];
            uy -= tau * vdy[it];
          }
          r = vr[it];
        }
        s_ux[k] = ux;
        s_uy[k] = uy;
        s_r[k] = r;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < EX * EY; e += BLOCK) {
      int ey = e / EX, ex = e % EX;
      int a = y0 - 1 + ey, b = x0 - 1 + ex;
      float cx[4] = {0, 0, 0, 0}, cy[4] = {0, 0, 0, 0};
      // one branch (not a chain of short-circuit branches, each re-zeroing the sums)
      const bool live = (ey < th + 1) & (ex < tw + 1) & (a >= 0) & (a < n - 1) & (b >= 0) &
                        (b < n - 1);
      if (live) {
        int k00 = ey * NX + ex;
        float ux[4] = {s_ux[k00], s_ux[k00 + 1], s_ux[k00 + NX], s_ux[k00 + NX + 1]};
        float uy[4] = {s_uy[k00], s_uy[k00 + 1], s_uy[k00 + NX], s_uy[k00 + NX + 1]};
        float rr[4] = {s_r[k00], s_r[k00 + 1], s_r[k00 + NX], s_r[k00 + NX + 1]};
        QuadField qux(ux), quy(uy), qr(rr);
        const unsigned base4 = (unsigned)mad24(a, n, b) << 2;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const float xi = q ? kGP1 : kGP0, eta = p ? kGP1 : kGP0;
            const float ps[4] = {(1.f - xi) * (1.f - eta), xi * (1.f - eta), (1.f - xi) * eta,
                                 xi * eta};
            float rq = qr.at(p, q);
            float gx, gy;
            float tv = sample_grad(T, T1, n4, base4, (float)(-b), (float)(n - 1 - b),
                                   (float)(-a), (float)(n - 1 - a), n - 2 - b, n - 2 - a,
                                   fmaf(qux.at(p, q), inv_h, xi), fmaf(quy.at(p, q), inv_h, eta),
                                   inv_h, &gx, &gy);
            float f = -w * (rq - ncc * (tv - mean) * inv_sig) * inv_sig;
            float fx = f * gx, fy = f * gy;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              cx[k] += ps[k] * fx;
              cy[k] += ps[k] * fy;
            }
          }
        }
        // lambda K_e u_e
        float kx[4], ky[4];
        ke_apply(ux, kx);
        ke_apply(uy, ky);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          cx[k] += lam * kx[k];
          cy[k] += lam * ky[k];
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        s_c[2 * k][e] = cx[k];
        s_c[2 * k + 1][e] = cy[k];
      }
    }
    __syncthreads();
    // rows of TX + 1 slots (a compile-time divisor); the slot past the tile's width is skipped
    constexpr int TW1 = TX + 1;
    for (int k = threadIdx.x; k < th * TW1; k += BLOCK) {
      int ty = k / TW1, tx = k - ty * TW1;
      if (tx >= tw) continue;
      int a = y0 + ty, b = x0 + tx;
      // elements (local coords): (ty, tx) is element (a-1, b-1) -> corner 3, etc.
      int e11 = ty * EX + tx, e10 = ty * EX + tx + 1, e01 = (ty + 1) * EX + tx,
          e00 = (ty + 1) * EX + tx + 1;
      float gx = (s_c[6][e11] + s_c[4][e10]) + (s_c[2][e01] + s_c[0][e00]);
      float gy = (s_c[7][e11] + s_c[5][e10]) + (s_c[3][e01] + s_c[1][e00]);
      unsigned o = (unsigned)mad24(a, n, b) << 2, og = (unsigned)mad24(a, gpi, b) << 2;
      int kn = (ty + 1) * NX + tx + 1;
      sto(G, og, gx);
      sto(G, gpn4 + og, gy);
      sto(un, o, s_ux[kn]);
      sto(un, nn4 + o, s_uy[kn]);
    }
    __syncthreads();
  }
}

// The gradient items of a step and its prolongations (slots that finished a level: disjoint
// from the gradient slots, and nothing here reads what they write), one item space made of
// the two lists in that order.
template <int TX, int TY>
__global__ void __launch_bounds__(BLOCK, LB_GRAD) k_grad(BatchDesc* D) {
  __shared__ GradLds<TX, TY> L;
  __shared__ int s_pos;
  const int ng = D->lists[WK_GRAD].total, np = D->lists[WK_PROLONG].total;
  const int total = ng + np;
  if (total <= 0) return;
  int chunk = (total + gridDim.x - 1) / gridDim.x;
  int b0 = placed_block<16>(chunk) * chunk, b1 = min(b0 + chunk, total);
  ItemCursor c;
  if (b0 < ng && cursor_range(D, WK_GRAD, b0, min(b1, ng), c, &s_pos)) {
    for (; c.item < c.end; ++c.item) {
      int s, t;
      cursor_slot(D, WK_GRAD, c, s, t);
      grad_item<TX, TY>(D, s, t, L);
    }
  }
  if (b1 > ng && cursor_range(D, WK_PROLONG, max(b0, ng) - ng, b1 - ng, c, &s_pos)) {
    for (; c.item < c.end; ++c.item) {
      int s, t;
      cursor_slot(D, WK_PROLONG, c, s, t);
      prolong_item(D, s, t);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Metric solve along one axis: S1 x = g on every line, S1 symmetric tridiagonal with the
// level's precomputed LU (a_i = -o / den_i, inv_den_i, c'_i). One wavefront solves one line:
// lane j holds nodes j*C .. j*C+C-1 in registers, composes the affine maps of the forward
// (y_i = a_i y_{i-1} + g_i / den_i) and backward (x_i = y_i - c'_i x_{i+1}) substitutions over
// its chunk, scans them across the 64 lanes with shuffles, and re-applies them.
// DIR 0: lines are columns of a strip staged in LDS (solve along y), reads G writes Z.
// DIR 1: lines are rows (solve along x), reads Z writes D, partial G.d and max |d|.

// Lane scans of the affine maps y -> A y + B of R lines across the 64 lanes of a wave, on DPP
// moves instead of LDS permutes: Hillis-Steele inside each row of 16 lanes (row_shr / row_shl),
// then across the rows (row broadcasts upward; lane reads of the row heads downward, which
// DPP has no broadcast for). A lane whose source is outside its row or masked off reads the
// identity (1, 0). The final one-lane shifts are wave_shr:1 / wave_shl:1.
template <int CTL, int ROWS, int R>
__device__ __forceinline__ void dpp_combine(float (&A)[R], float (&B)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    float Ap = __builtin_amdgcn_update_dpp(1.f, A[r], CTL, ROWS, 0xf, false);
    float Bp = __builtin_amdgcn_update_dpp(0.f, B[r], CTL, ROWS, 0xf, false);
    B[r] = fmaf(A[r], Bp, B[r]);
    A[r] = A[r] * Ap;
  }
}
__device__ __forceinline__ float lane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
// Inclusive scan from lane 0 (lane i ends with lanes 0..i composed, later lanes outermost).
template <int R>
__device__ __forceinline__ void scan_up(float (&A)[R], float (&B)[R]) {
  dpp_combine<0x111, 0xf>(A, B);  // row_shr:1
  dpp_combine<0x112, 0xf>(A, B);  // row_shr:2
  dpp_combine<0x114, 0xf>(A, B);  // row_shr:4
  dpp_combine<0x118, 0xf>(A, B);  // row_shr:8
  dpp_combine<0x142, 0xa>(A, B);  // row_bcast:15 into rows 1 and 3
  dpp_combine<0x143, 0xc>(A, B);  // row_bcast:31 into rows 2 and 3
}
// Inclusive scan from lane 63 (lane i ends with lanes i..63 composed).
template <int R>
__device__ __forceinline__ void scan_down(float (&A)[R], float (&B)[R], int lane) {
  dpp_combine<0x101, 0xf>(A, B);  // row_shl:1
  dpp_combine<0x102, 0xf>(A, B);  // row_shl:2
  dpp_combine<0x104, 0xf>(A, B);  // row_shl:4
  dpp_combine<0x108, 0xf>(A, B);  // row_shl:8
  int row = lane >> 4;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    // row aggregates from the first lane of each row; the maps of the rows after a row
    float a1 = lane_f(A[r], 16), b1 = lane_f(B[r], 16);
    float a2 = lane_f(A[r], 32), b2 = lane_f(B[r], 32);
    float a3 = lane_f(A[r], 48), b3 = lane_f(B[r], 48);
    float t2a = a2 * a3, t2b = fmaf(a2, b3, b2);
    float t1a = a1 * t2a, t1b = fmaf(a1, t2b, b1);
    float ta = row == 0 ? t1a : row == 1 ? t2a : row == 2 ? a3 : 1.f;
    float tb = row == 0 ? t1b : row == 1 ? t2b : row == 2 ? b3 : 0.f;
    B[r] = fmaf(A[r], tb, B[r]);
    A[r] = A[r] * ta;
  }
}

// Levels have n = 2^l + 1 nodes, so the C chosen for a level (the smallest of 1, 2, 3, 5, 9, 17
// with 64 C >= n) gives exactly coef_pitch(n) = 64 C node slots per line. The coefficient
// arrays are zero past node n - 1, so every lane runs its whole chunk without a branch: a
// padded node's forward map is the constant 0 (its y is 0) and, in the backward direction,
// c'_{n-1} = 0 already cuts node n - 1 off from anything above it.
template <int R, int C>
__device__ __forceinline__ void solve_lines(float (&v)[R][C], int n, int lane,
                                            const float* __restrict__ coef) {
  const int cs = coef_pitch(n);
  const GAS float* ca = (const GAS float*)coef;  // a_i
  const GAS float* ci = ca + cs;                  // 1 / den_i
  const GAS float* cp = ca + 2 * cs;              // c'_i
  int base = lane * C;
  float A[R], B[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    A[r] = 1.f;
    B[r] = 0.f;
  }
#pragma unroll
  for (int k = 0; k < C; ++k) {
    int i = base + k;
    float a = ca[i], c = ci[i];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      A[r] = a * A[r];
      B[r] = fmaf(a, B[r], c * v[r][k]);
    }
  }
  float y[R];
  scan_up<R>(A, B);
#pragma unroll
  for (int r = 0; r < R; ++r) y[r] = __builtin_amdgcn_update_dpp(0.f, B[r], 0x138, 0xf, 0xf, false);
#pragma unroll
  for (int k = 0; k < C; ++k) {
    int i = base + k;
    float a = ca[i], c = ci[i];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      y[r] = fmaf(a, y[r], c * v[r][k]);
      v[r][k] = y[r];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    A[r] = 1.f;
    B[r] = 0.f;
  }
#pragma unroll
  for (int k = C - 1; k >= 0; --k) {
    int i = base + k;
    float mm = -cp[i];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      A[r] = mm * A[r];
      B[r] = fmaf(mm, B[r], v[r][k]);
    }
  }
  scan_down<R>(A, B, lane);
#pragma unroll
  for (int r = 0; r < R; ++r) y[r] = __builtin_amdgcn_update_dpp(0.f, B[r], 0x130, 0xf, 0xf, false);
#pragma unroll
  for (int k = C - 1; k >= 0; --k) {
    int i = base + k;
    float mm = -cp[i];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      y[r] = fmaf(mm, y[r], v[r][k]);
      v[r][k] = y[r];
    }
  }
}

// Orders LDS accesses of one wavefront (lanes exchange data through LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lines solved together by one wavefront for C nodes per lane (LDS per wave stays <= 10 KB).
#define SM_R9 4
template <int C>
struct SmoothR {
  static constexpr int value = C <= 9 ? SM_R9 : 2;
};

// One smoother item: lines [line0, line0 + nl) of one component.
template <int DIR, int C>
__device__ __forceinline__ void smooth_item(const float* src, float* dst, const float* Gp,
                                            const float* coef, int n, int P, int line0, int nl,
                                            int SL, float* s_buf, double& gd, double& dm) {
  constexpr int R = SmoothR<C>::value;
  constexpr int NW = BLOCK / 64;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float v[R][C];
  if (DIR == 0) {
    // strip [n][SL] with pitch SL + 1; wave wv solves columns g .. g+R-1, g = R wv + R NW j.
    // SL is a power of two (8, 16 or 32): strip element k is row k >> sh, line k & (SL - 1).
    int pitch = SL + 1;
    const int sh = __builtin_ctz(SL);
    {
      // UB loads per lane in flight before the LDS stores (indices clamped into the strip);
      // 17 covers a 513-node strip of 16 lines in two rounds
#define SM_UB 17
      constexpr int UB = SM_UB;
      const int tot = n << sh;
      const GAS float* sb = (const GAS float*)src + line0;
      for (int k0 = threadIdx.x; k0 < tot; k0 += UB * BLOCK) {
        float v[UB];
#pragma unroll
        for (int j = 0; j < UB; ++j) {
          int k = min(k0 + j * BLOCK, tot - 1);
          int i = k >> sh, L = min(k & (SL - 1), nl - 1);
          v[j] = sb[(unsigned)(i * P + L)];
        }
#pragma unroll
        for (int j = 0; j < UB; ++j) {
          int k = k0 + j * BLOCK;
          if (k < tot) {
            int i = k >> sh, L = k & (SL - 1);
            s_buf[i * pitch + L] = L < nl ? v[j] : 0.f;
          }
        }
      }
    }
    __syncthreads();
    for (int g = wv * R; g < nl; g += R * NW) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < C; ++k) {
          int i = lane * C + k, L = min(g + r, SL - 1);
          float x = s_buf[min(i, n - 1) * pitch + L];
          v[r][k] = i < n ? x : 0.f;
        }
      solve_lines<R, C>(v, n, lane, coef);
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < C; ++k) {
          int i = lane * C + k;
          if (i < n && g + r < nl) s_buf[i * pitch + g + r] = v[r][k];
        }
    }
    __syncthreads();
    GAS float* db = (GAS float*)dst + line0;
    for (int k = threadIdx.x; k < (n << sh); k += BLOCK) {
      int i = k >> sh, L = k & (SL - 1);
      if (L < nl) db[(unsigned)(i * P + L)] = s_buf[i * pitch + L];
    }
  } else {
    // each wave stages R rows in its own LDS area (row pitch 64 C + 1)
    int pitch = 64 * C + 1;
    float* rows = s_buf + wv * R * pitch;
    float dmf = 0.f;  // max |d| (exact in FP32)
    for (int g = wv * R; g < nl; g += R * NW) {
      int nr = min(R, nl - g);
      if constexpr (C <= 9) {
        // all R x C loads of a lane in flight before the LDS stores (indices clamped)
        float t[R][C];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k = 0; k < C; ++k) {
            int i = min(lane + 64 * k, n - 1);
            const float* sr = src + (size_t)(line0 + g + min(r, nr - 1)) * P;
            t[r][k] = gld(sr, i);
          }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int k = 0; k < C; ++k) {
            int i = lane + 64 * k;
            if (r < nr && i < n) rows[r * pitch + i] = t[r][k];
          }
      } else {
        for (int r = 0; r < nr; ++r) {
          const float* sr = src + (size_t)(line0 + g + r) * P;
          for (int i = lane; i < n; i += 64) rows[r * pitch + i] = gld(sr, i);
        }
      }
      wave_sync();
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < C; ++k) {
          int i = lane * C + k;
          v[r][k] = (i < n && r < nr) ? rows[r * pitch + i] : 0.f;
        }
      wave_sync();
      solve_lines<R, C>(v, n, lane, coef);
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < C; ++k) {
          int i = lane * C + k;
          if (i < n && r < nr) rows[r * pitch + i] = v[r][k];
        }
      wave_sync();
      // the C loads of G of a row in flight together
      for (int r = 0; r < nr; ++r) {
        float* dr = dst + (size_t)(line0 + g + r) * n;
        const float* gr = Gp + (size_t)(line0 + g + r) * P;
        float t[C];
#pragma unroll
        for (int k = 0; k < C; ++k) t[k] = gld(gr, min(lane + 64 * k, n - 1));
#pragma unroll
        for (int k = 0; k < C; ++k) {
          int i = lane + 64 * k;
          if (i < n) {
            float x = rows[r * pitch + i];
            gst(dr, i, x);
            gd += (double)(t[k] * x);
            dmf = fmaxf(dmf, fabsf(x));
          }
        }
      }
      wave_sync();
    }
    dm = fmax(dm, (double)dmf);
  }
}

// BIG: the instance that also handles lines of more than 576 nodes (17 per lane); the smaller
// instance leaves that path out, which keeps its register allocation free of spills. The host
// launches BIG only when the batch's finest level needs it.
#define LB_SMX LB_SMOOTH
template <int DIR, bool BIG>
__global__ void __launch_bounds__(BLOCK, DIR ? LB_SMX : LB_SMOOTH) k_smooth(BatchDesc* D) {
  extern __shared__ float s_buf[];
  __shared__ double s_red[(BLOCK / 64) * 2];
  __shared__ int s_pos;
  const int kind = DIR ? WK_SMX : WK_SMY;
  ItemCursor c;
  // column strips: a strip of 16 lines reads and writes one half of each 128-byte line, its
  // neighbour the other half
  if (!cursor_begin<DIR ? 0 : 16>(D, kind, c, &s_pos)) return;
  for (; c.item < c.end; ++c.item) {
    int s, t;
    cursor_slot(D, kind, c, s, t);
    const SlotState* stp = D->state + s;
    if (stp->phase != PH_GRAD) continue;
    int l = stp->level;
    int n = lvl_n(l);
    size_t nn = (size_t)n * n;
    const LevelGeom& g = D->geom[l];
    int SL = g.sm_lines;
    int comp = t / g.sm_items;
    int line0 = (t % g.sm_items) * SL;
    int nl = min(SL, n - line0);
    const int P = row_pitch(n);
    const size_t np = (size_t)n * P;
    const float* src = (DIR ? D->zbuf : D->gbuf) + (size_t)s * D->slot_p_stride + comp * np;
    float* dst = DIR ? D->dbuf + (size_t)s * D->slot_f_stride + comp * nn
                     : D->zbuf + (size_t)s * D->slot_p_stride + comp * np;
    const float* Gp = D->gbuf + (size_t)s * D->slot_p_stride + comp * np;
    const float* coef = D->coef + g.coef_off;
    double gd = 0.0, dm = 0.0;
    __syncthreads();
    int Cn = (n + 63) / 64;
    if (Cn <= 1) smooth_item<DIR, 1>(src, dst, Gp, coef, n, P, line0, nl, SL, s_buf, gd, dm);
    else if (Cn <= 2) smooth_item<DIR, 2>(src, dst, Gp, coef, n, P, line0, nl, SL, s_buf, gd, dm);
    else if (Cn <= 3) smooth_item<DIR, 3>(src, dst, Gp, coef, n, P, line0, nl, SL, s_buf, gd, dm);
    else if (Cn <= 5) smooth_item<DIR, 5>(src, dst, Gp, coef, n, P, line0, nl, SL, s_buf, gd, dm);
    else if (Cn <= 9) smooth_item<DIR, 9>(src, dst, Gp, coef, n, P, line0, nl, SL, s_buf, gd, dm);
    else if constexpr (BIG) smooth_item<DIR, 17>(src, dst, Gp, coef, n, P, line0, nl, SL, s_buf, gd, dm);
    if (DIR == 1) {
      double acc[2] = {gd, dm};
      block_sum<2>(acc, s_red, true);
      if (threadIdx.x == 0) {
        double* pr = slot_partial(D, s, kind, t);
        pr[0] = acc[0];
        pr[1] = acc[1];
      }
    }
  }
}

// Windowed metric solve: d = (S1^-1 (x) S1^-1) G for one SW_T x SW_T tile of one component in
// one pass. The LU recurrences of S1 contract by a factor rho(beta) per node (0.35 for
// beta = 1), so a node's solution depends on G within a few nodes only: each tile solves the
// columns of its window (tile plus H nodes of halo on every side, clipped to the domain, with
// the LU coefficients of the global rows) and then the rows of its output nodes. The host picks
// H with rho^H below FP32 resolution; where the window reaches the domain edge the solve is the
// exact one. Reads G once (halo re-reads hit the cache) and writes d: 16 B per node instead of
// the 40 of two full passes through an intermediate. Partials: G.d and max |d| per tile.
template <int H>
__global__ void __launch_bounds__(SW_THREADS) k_smooth_win(BatchDesc* D) {
  constexpr int WM = SW_T + 1 + 2 * H;  // largest window extent (last tile holds SW_T + 1)
  constexpr int PITCH = WM + 1;
  __shared__ float s[WM * PITCH];
  __shared__ double s_red[2][SW_THREADS / 64];
  __shared__ int s_pos;
  const int tid = threadIdx.x;
  ItemCursor c;
  if (!cursor_begin(D, WK_SMX, c, &s_pos)) return;
  for (; c.item < c.end; ++c.item) {
    int sl, t;
    cursor_slot(D, WK_SMX, c, sl, t);
    const SlotState* stp = D->state + sl;
    if (stp->phase != PH_GRAD) continue;
    int l = stp->level;
    int n = lvl_n(l);
    size_t nn = (size_t)n * n;
    const LevelGeom& g = D->geom[l];
    int nt = g.sw_tiles;
    int comp = t / (nt * nt), tile = t - comp * nt * nt;
    int ty = tile / nt, tx = tile - ty * nt;
    int oy0 = ty * SW_T, oy1 = ty == nt - 1 ? n : oy0 + SW_T;
    int ox0 = tx * SW_T, ox1 = tx == nt - 1 ? n : ox0 + SW_T;
    int wy0 = max(0, oy0 - H), wy1 = min(n, oy1 + H);
    int wx0 = max(0, ox0 - H), wx1 = min(n, ox1 + H);
    int hy = wy1 - wy0, hx = wx1 - wx0;
    const int P = row_pitch(n);
    const float* G = D->gbuf + (size_t)sl * D->slot_p_stride + comp * (size_t)n * P;
    float* dst = D->dbuf + (size_t)sl * D->slot_f_stride + comp * nn;
    const float* ca = D->coef + g.coef_off;  // a_i
    const float* ci = ca + coef_pitch(n);    // 1 / den_i
    const float* cp = ca + 2 * coef_pitch(n);  // c'_i
    __syncthreads();
    for (int k = tid; k < hy * hx; k += SW_THREADS) {
      int r = k / hx, q = k - r * hx;
      s[r * PITCH + q] = G[(size_t)(wy0 + r) * P + wx0 + q];
    }
    __syncthreads();
    if (tid < hx) {  // column tid of the window, rows wy0 .. wy1 - 1
      float v[WM];
#pragma unroll
      for (int r = 0; r < WM; ++r) v[r] = r < hy ? s[r * PITCH + tid] : 0.f;
      float y = 0.f;
#pragma unroll
      for (int r = 0; r < WM; ++r)
        if (r < hy) {
          int i = wy0 + r;
          y = fmaf(ca[i], y, ci[i] * v[r]);
          v[r] = y;
        }
      float x = 0.f;
#pragma unroll
      for (int r = WM - 1; r >= 0; --r)
        if (r < hy) {
          int i = wy0 + r;
          x = fmaf(-cp[i], x, v[r]);
          v[r] = x;
        }
#pragma unroll
      for (int r = 0; r < WM; ++r)
        if (r < hy) s[r * PITCH + tid] = v[r];
    }
    __syncthreads();
    int rows = oy1 - oy0, cols = ox1 - ox0;
    if (tid < rows) {  // output row tid, columns wx0 .. wx1 - 1
      float* row = s + (oy0 - wy0 + tid) * PITCH;
      float v[WM];
#pragma unroll
      for (int q = 0; q < WM; ++q) v[q] = q < hx ? row[q] : 0.f;
      float y = 0.f;
#pragma unroll
      for (int q = 0; q < WM; ++q)
        if (q < hx) {
          int i = wx0 + q;
          y = fmaf(ca[i], y, ci[i] * v[q]);
          v[q] = y;
        }
      float x = 0.f;
#pragma unroll
      for (int q = WM - 1; q >= 0; --q)
        if (q < hx) {
          int i = wx0 + q;
          x = fmaf(-cp[i], x, v[q]);
          v[q] = x;
        }
#pragma unroll
      for (int q = 0; q < WM; ++q)
        if (q < hx) row[q] = v[q];
    }
    __syncthreads();
    double gd = 0.0, dm = 0.0;
    for (int k = tid; k < rows * cols; k += SW_THREADS) {
      int j = k / cols, q = k - j * cols;
      float xv = s[(oy0 - wy0 + j) * PITCH + (ox0 - wx0) + q];
      size_t gi = (size_t)(oy0 + j) * n + ox0 + q;
      dst[gi] = xv;
      gd += (double)(G[(size_t)(oy0 + j) * P + ox0 + q] * xv);
      dm = fmax(dm, (double)fabsf(xv));
    }
    gd = wave_sum(gd);
    dm = wave_max(dm);
    if ((tid & 63) == kTotalLane) {
      s_red[0][tid >> 6] = gd;
      s_red[1][tid >> 6] = dm;
    }
    __syncthreads();
    if (tid == 0) {
      double a = s_red[0][0], b = s_red[1][0];
      for (int w = 1; w < SW_THREADS / 64; ++w) {
        a += s_red[0][w];
        b = fmax(b, s_red[1][w]);
      }
      double* pr = slot_partial(D, sl, WK_SMX, t);
      pr[0] = a;
      pr[1] = b;
    }
  }
}

// Per-slot finalisation of the metric solve: G.d, max |d|, step bound and first ladder top.
__global__ void __launch_bounds__(BLOCK) k_smooth_fin(BatchDesc* D) {
  __shared__ double s_red[(BLOCK / 64) * 2];
  const WorkList wl = D->lists[WK_SMX];
  const int* off = D->list_off + (size_t)WK_SMX * (D->max_slots + 1);
  for (int pos = blockIdx.x; pos < wl.n_slots; pos += gridDim.x) {
    // listed slots are in GRAD (nothing between the plan and here changes a phase); the item
    // count comes from the list offsets, so the partial loads do not wait for the slot state
    int s = D->list_slots[(size_t)WK_SMX * D->max_slots + pos];
    SlotState* stp = D->state + s;
    SlotState st;
    load_head(st, *stp);  // in flight with the partial loads
    double tot[2];
    partials_local<2>(D, s, WK_SMX, off[pos + 1] - off[pos], tot, true);
    // the node counters (only this workgroup writes them) and the run's parameters load while
    // the partials reduce, instead of after the first store
    long long* nc_s = D->node_count + (size_t)s * WK_COUNT;
    long long nodes[3];
    double step_cap, tau_min_rel;
    int ladder_k, halo;
    if (threadIdx.x == 0) {
      nodes[0] = nc_s[WK_GRAD];
      nodes[1] = nc_s[WK_SMY];
      nodes[2] = nc_s[WK_SMX];
      step_cap = D->step_cap;
      tau_min_rel = D->tau_min_rel;
      ladder_k = D->ladder_k;
      halo = D->smooth_halo;
    }
    block_sum<2>(tot, s_red, true);
    if (threadIdx.x == 0) {
      int l = st.level;
      int n = lvl_n(l);
      nc_s[WK_GRAD] = nodes[0] + (long long)n * n;
      if (!halo) nc_s[WK_SMY] = nodes[1] + (long long)n * n;
      nc_s[WK_SMX] = nodes[2] + (long long)n * n;
      st.ub ^= 1;          // the gradient kernel wrote u - tau_pend d to the other buffer
      st.tau_pend = 0.0;
      st.gtd = tot[0];
      st.dmax = tot[1];
      if (!(st.gtd > 0.0) || !(st.dmax > 0.0)) {
        level_done(st);
      } else {
        double h = 1.0 / (n - 1);
        st.tau_max = step_cap * h / st.dmax;
        st.top = fmin(ldexp(st.tau_prev, ladder_k), st.tau_max);
        st.rung = 0;
        // a line search whose first step is already below tau_min_rel * tau_max is not begun
        if (st.top < tau_min_rel * st.tau_max) level_done(st);
        else st.phase = PH_LADDER;
      }
      store_head(*stp, st);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// Setup / finish kernels (one launch per batch)

// Full-weighting restriction of planes: dst(A,B) = sum w_p w_q src(2A+p, 2B+q) / sum w over
// in-range fine nodes. Plane p lives at base + (p / inner) * outer + (p % inner) * innerst.
__global__ void __launch_bounds__(BLOCK) k_restrict(const float* src, long long s_outer,
                                                    long long s_inner, float* dst,
                                                    long long d_outer, long long d_inner,
                                                    int inner, int nf, int planes) {
  int nc = (nf - 1) / 2 + 1;
  long long total = (long long)planes * nc * nc;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < total;
       k += (long long)gridDim.x * BLOCK) {
    int p = (int)(k / ((long long)nc * nc));
    int rem = (int)(k % ((long long)nc * nc));
    int A = rem / nc, B = rem % nc;
    const float* f = src + (p / inner) * s_outer + (p % inner) * s_inner;
    float sum = 0.f, ws = 0.f;
    for (int dp = -1; dp <= 1; ++dp) {
      int a = 2 * A + dp;
      if (a < 0 || a >= nf) continue;
      float wa = dp == 0 ? 2.f : 1.f;
      float row = 0.f, rw = 0.f;
      for (int dq = -1; dq <= 1; ++dq) {
        int b = 2 * B + dq;
        if (b < 0 || b >= nf) continue;
        float wb = dq == 0 ? 2.f : 1.f;
        row = fmaf(wb, f[(size_t)a * nf + b], row);
        rw += wb;
      }
      sum = fmaf(wa, row, sum);
      ws += wa * rw;
    }
    dst[(p / inner) * d_outer + (p % inner) * d_inner + (size_t)A * nc + B] = sum / ws;
  }
}

// Pixel frames [N][H][W] (H == 2^L or 2^L + 1) -> nodal grids [N][n][n], replicating the last
// row/column when H == 2^L. scale multiplies every value.
__global__ void __launch_bounds__(BLOCK) k_to_nodes(const float* src, int H, long long s_plane,
                                                    float* dst, int n, long long d_plane,
                                                    int planes, float scale) {
  long long total = (long long)planes * n * n;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < total;
       k += (long long)gridDim.x * BLOCK) {
    int p = (int)(k / ((long long)n * n));
    int rem = (int)(k % ((long long)n * n));
    int a = min(rem / n, H - 1), b = min(rem % n, H - 1);
    dst[p * d_plane + rem] = scale * src[p * s_plane + (size_t)a * H + b];
  }
}

// Nodal [planes][n][n] -> pixels [planes][H][H] (crop), times scale.
__global__ void __launch_bounds__(BLOCK) k_from_nodes(const float* src, int n, long long s_plane,
                                                      float* dst, int H, long long d_plane,
                                                      int planes, float scale) {
  long long total = (long long)planes * H * H;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < total;
       k += (long long)gridDim.x * BLOCK) {
    int p = (int)(k / ((long long)H * H));
    int rem = (int)(k % ((long long)H * H));
    int a = rem / H, b = rem % H;
    dst[p * d_plane + rem] = scale * src[p * s_plane + (size_t)a * n + b];
  }
}

__global__ void __launch_bounds__(BLOCK) k_fill_strided(float* p, long long outer, long long per,
                                                        int n_outer, float v) {
  long long total = (long long)n_outer * per;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < total;
       k += (long long)gridDim.x * BLOCK)
    p[(k / per) * outer + (k % per)] = v;
}

// Bilinear coefficients of each node of N frames of n x n nodes: v, the difference to the node
// to the right, to the node below, and the cross difference (v11 - v10) - (v01 - v00); the
// differences that would leave the frame are 0 (a sample there has fraction 0 on that axis).
__global__ void __launch_bounds__(BLOCK) k_tcoef(const float* f, int n, long long total,
                                                 float4* coef) {
  const long long nn = (long long)n * n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    int r = (int)(i % nn);
    int a = r / n, b = r - a * n;
    float v00 = f[i];
    bool rx = b < n - 1, ry = a < n - 1;
    float v01 = rx ? f[i + 1] : v00, v10 = ry ? f[i + n] : v00;
    float v11 = rx && ry ? f[i + n + 1] : v00;
    float c1 = rx ? v01 - v00 : 0.f, c2 = ry ? v10 - v00 : 0.f;
    float c3 = rx && ry ? (v11 - v10) - (v01 - v00) : 0.f;
    coef[i] = make_float4(v00, c1, c2, c3);
  }
}

__global__ void __launch_bounds__(BLOCK) k_fill(float* p, long long count, float v) {
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < count;
       k += (long long)gridDim.x * BLOCK)
    p[k] = v;
}

// Element sums of planes for normalisation: per (plane, row band) partials of
// S1 = sum_e h^2/4 sum_corners F and S2 = sum_e F_e^T M_e F_e (FP64).
__global__ void __launch_bounds__(BLOCK) k_elem_sums(const float* src, long long plane_stride,
                                                     int n, int bands, double* partial) {
  __shared__ double s_red[(BLOCK / 64) * 2];
  int p = blockIdx.x / bands, band = blockIdx.x % bands;
  const float* f = src + p * plane_stride;
  int ne = n - 1;
  int rows = (ne + bands - 1) / bands;
  int a0 = band * rows, a1 = min(a0 + rows, ne);
  double h2 = 1.0 / ((double)ne * ne);
  double s1 = 0.0, s2 = 0.0;
  for (int a = a0; a < a1; ++a)
    for (int b = threadIdx.x; b < ne; b += BLOCK) {
      double f0 = f[(size_t)a * n + b], f1 = f[(size_t)a * n + b + 1];
      double f2 = f[(size_t)(a + 1) * n + b], f3 = f[(size_t)(a + 1) * n + b + 1];
      s1 += (f0 + f1 + f2 + f3);
      double sq = f0 * f0 + f1 * f1 + f2 * f2 + f3 * f3;
      double edge = f0 * f1 + f0 * f2 + f1 * f3 + f2 * f3;
      double opp = f0 * f3 + f1 * f2;
      s2 += 4.0 * sq + 4.0 * edge + 2.0 * opp;
    }
  double acc[2] = {s1 * h2 * 0.25, s2 * h2 / 36.0};
  block_sum<2>(acc, s_red);
  if (threadIdx.x == 0) {
    partial[(size_t)blockIdx.x * 2] = acc[0];
    partial[(size_t)blockIdx.x * 2 + 1] = acc[1];
  }
}

// Per plane: mean = S1, sigma = sqrt(S2 - S1^2) from the band partials (fixed order).
// mode 0: writes mean/sigma to ms[2 * p]; mode 1: writes S1 to rsum[p * rs_stride + rs_off].
__global__ void k_elem_final(const double* partial, int bands, int planes, int mode, double* ms,
                             double* rsum, int rs_stride, int rs_off) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= planes) return;
  double s1 = 0.0, s2 = 0.0;
  for (int b = 0; b < bands; ++b) {
    s1 += partial[((size_t)p * bands + b) * 2];
    s2 += partial[((size_t)p * bands + b) * 2 + 1];
  }
  if (mode == 0) {
    double var = s2 - s1 * s1;
    ms[2 * p] = s1;
    ms[2 * p + 1] = var > 0.0 ? sqrt(var) : 0.0;
  } else {
    rsum[(size_t)p * rs_stride + rs_off] = s1;
  }
}

// F <- (F - mean) / sigma per plane (sigma == 0 leaves the plane, the host reports EINVAL).
__global__ void __launch_bounds__(BLOCK) k_normalize(float* f, long long plane_stride,
                                                     long long per_plane, int planes,
                                                     const double* ms) {
  long long total = (long long)planes * per_plane;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < total;
       k += (long long)gridDim.x * BLOCK) {
    int p = (int)(k / per_plane);
    long long i = k % per_plane;
    double m = ms[2 * p], sg = ms[2 * p + 1];
    if (sg > 0.0) f[p * plane_stride + i] = (float)((f[p * plane_stride + i] - m) / sg);
  }
}

// Composition (phi_jk o phi_ij): w = u_ij + u_jk(x + u_ij), clamped bilinear, domain units.
// For op k: left = elems + left_idx[k] * estride, right = elems + right_idx[k] * estride,
// out = out_base + k * ostride. Index -1 means "use the explicit pointer" (single op).
__global__ void __launch_bounds__(BLOCK) k_compose(const float* elems, long long estride,
                                                   const int* left_idx, const int* right_idx,
                                                   float* out_base, long long ostride, int n,
                                                   int ops) {
  size_t nn = (size_t)n * n;
  long long total = (long long)ops * nn;
  float inv_h = (float)(n - 1);
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < total;
       k += (long long)gridDim.x * BLOCK) {
    int op = (int)(k / nn);
    int i = (int)(k % nn);
    const float* ul = elems + left_idx[op] * estride;
    const float* ur = elems + right_idx[op] * estride;
    float* w = out_base + op * ostride;
    int a = i / n, b = i % n;
    float ux = ul[i], uy = ul[nn + i];
    float tx = ux * inv_h, ty = uy * inv_h;
    float vx = sample_bil<false>(ur, n, b, tx, a, ty, inv_h, nullptr, nullptr);
    float vy = sample_bil<false>(ur + nn, n, b, tx, a, ty, inv_h, nullptr, nullptr);
    w[i] = ux + vx;
    w[nn + i] = uy + vy;
  }
}

// Finished slots: element[out_idx[s]] = u_L[ub] - tau_pend d.
__global__ void __launch_bounds__(BLOCK) k_finish(BatchDesc* D, const int* out_idx,
                                                  float* elems, long long estride) {
  int L = D->finest;
  int n = lvl_n(L);
  size_t per = 2 * (size_t)n * n;
  long long total = (long long)D->n_slots * per;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < total;
       k += (long long)gridDim.x * BLOCK) {
    int s = (int)(k / per);
    size_t i = k % per;
    const SlotState& st = D->state[s];
    if (st.level != L) continue;  // aborted before the finest level: leave the element
    const float* u = slot_u(D, s, L, st.ub);
    const float* d = D->dbuf + (size_t)s * D->slot_f_stride;
    float tau = (float)st.tau_pend;
    elems[out_idx[s] * estride + i] = tau != 0.f ? u[i] - tau * d[i] : u[i];
  }
}

// ------------------------------------------------------------------------------------------
// Slot-pool kernels: a registration is started in whichever slot is free, so these address
// slots through index lists (slots[k] is the slot of the k-th listed registration).

// D->state[slots[k]] = staged[k]; the slots' node counters restart at zero.
__global__ void __launch_bounds__(BLOCK) k_pool_assign(BatchDesc* D, const SlotState* staged,
                                                       const int* slots, int ops) {
  constexpr int W = sizeof(SlotState) / 4;
  long long total = (long long)ops * W;
  for (long long i = blockIdx.x * (long long)BLOCK + threadIdx.x; i < total;
       i += (long long)gridDim.x * BLOCK) {
    int k = (int)(i / W), w = (int)(i % W);
    reinterpret_cast<int*>(D->state + slots[k])[w] = reinterpret_cast<const int*>(staged + k)[w];
  }
  for (long long i = blockIdx.x * (long long)BLOCK + threadIdx.x; i < (long long)ops * WK_COUNT;
       i += (long long)gridDim.x * BLOCK)
    D->node_count[(size_t)slots[i / WK_COUNT] * WK_COUNT + i % WK_COUNT] = 0;
}

// Identity start: both components of listed slots' first u buffer on level l are zero.
__global__ void __launch_bounds__(BLOCK) k_pool_zero(BatchDesc* D, int l, const int* slots,
                                                     int ops) {
  int n = lvl_n(l);
  long long per = 2LL * n * n;
  for (long long i = blockIdx.x * (long long)BLOCK + threadIdx.x; i < (long long)ops * per;
       i += (long long)gridDim.x * BLOCK)
    slot_u(D, slots[i / per], l, 0)[i % per] = 0.f;
}

// Composition start on level L: the level-L u of slot slots[k] = (vbuf + off1[k]) (.)
// (vbuf + off0[k]) (w = u_ij + u_jk(x + u_ij), clamped bilinear, domain units).
__global__ void __launch_bounds__(BLOCK) k_pool_compose(BatchDesc* D, int L, const float* vbuf,
                                                        const long long* off0,
                                                        const long long* off1, const int* slots,
                                                        int ops) {
  int n = lvl_n(L);
  size_t nn = (size_t)n * n;
  float inv_h = (float)(n - 1);
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < (long long)ops * nn;
       k += (long long)gridDim.x * BLOCK) {
    int op = (int)(k / nn);
    int i = (int)(k % nn);
    const float* ul = vbuf + off0[op];
    const float* ur = vbuf + off1[op];
    float* w = slot_u(D, slots[op], L, 0);
    int a = i / n, b = i % n;
    float ux = ul[i], uy = ul[nn + i];
    float tx = ux * inv_h, ty = uy * inv_h;
    float vx = sample_bil<false>(ur, n, b, tx, a, ty, inv_h, nullptr, nullptr);
    float vy = sample_bil<false>(ur + nn, n, b, tx, a, ty, inv_h, nullptr, nullptr);
    w[i] = ux + vx;
    w[nn + i] = uy + vy;
  }
}

// Full-weighting restriction of listed slots' first u buffer from level l to level l - 1.
__global__ void __launch_bounds__(BLOCK) k_pool_restrict(BatchDesc* D, int l, const int* slots,
                                                         int ops) {
  int nf = lvl_n(l), nc = lvl_n(l - 1);
  long long per = (long long)nc * nc;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < (long long)ops * 2 * per;
       k += (long long)gridDim.x * BLOCK) {
    int p = (int)(k / per), rem = (int)(k % per);
    int op = p >> 1, comp = p & 1;
    int A = rem / nc, B = rem % nc;
    const float* f = slot_u(D, slots[op], l, 0) + (size_t)comp * nf * nf;
    float sum = 0.f, ws = 0.f;
    for (int dp = -1; dp <= 1; ++dp) {
      int a = 2 * A + dp;
      if (a < 0 || a >= nf) continue;
      float wa = dp == 0 ? 2.f : 1.f;
      float row = 0.f, rw = 0.f;
      for (int dq = -1; dq <= 1; ++dq) {
        int b = 2 * B + dq;
        if (b < 0 || b >= nf) continue;
        float wb = dq == 0 ? 2.f : 1.f;
        row = fmaf(wb, f[(size_t)a * nf + b], row);
        rw += wb;
      }
      sum = fmaf(wa, row, sum);
      ws += wa * rw;
    }
    slot_u(D, slots[op], l - 1, 0)[(size_t)comp * nc * nc + (size_t)A * nc + B] = sum / ws;
  }
}

// Staged guesses on level l (src + src_idx[k] * sstride, [2][n_l^2]) into listed slots.
__global__ void __launch_bounds__(BLOCK) k_pool_copy(BatchDesc* D, int l, const float* src,
                                                     long long sstride, const int* src_idx,
                                                     const int* slots, int ops) {
  int n = lvl_n(l);
  long long per = 2LL * n * n;
  for (long long i = blockIdx.x * (long long)BLOCK + threadIdx.x; i < (long long)ops * per;
       i += (long long)gridDim.x * BLOCK) {
    int k = (int)(i / per);
    slot_u(D, slots[k], l, 0)[i % per] = src[src_idx[k] * sstride + i % per];
  }
}

// Resumed results: the first u buffer of level l of slot slots[k] = vbuf + offs[k] ([2][n][n]).
__global__ void __launch_bounds__(BLOCK) k_pool_copy_off(BatchDesc* D, int l, const float* vbuf,
                                                         const long long* offs, const int* slots,
                                                         int ops) {
  int n = lvl_n(l);
  long long per = 2LL * n * n;
  for (long long i = blockIdx.x * (long long)BLOCK + threadIdx.x; i < (long long)ops * per;
       i += (long long)gridDim.x * BLOCK) {
    int k = (int)(i / per);
    slot_u(D, slots[k], l, 0)[i % per] = vbuf[offs[k] + i % per];
  }
}

// Finished listed slots whose finest level is L: vbuf + outs[k] = u_L[ub] - tau_pend d of slot
// slots[k] (a slot that stopped before level L leaves its output untouched).
__global__ void __launch_bounds__(BLOCK) k_pool_finish(BatchDesc* D, int L, const int* slots,
                                                       const long long* outs, int ops,
                                                       float* vbuf) {
  int n = lvl_n(L);
  size_t per = 2 * (size_t)n * n;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < (long long)ops * per;
       k += (long long)gridDim.x * BLOCK) {
    int op = (int)(k / per);
    size_t i = k % per;
    int s = slots[op];
    const SlotState& st = D->state[s];
    if (st.level != L) continue;
    const float* u = slot_u(D, s, L, st.ub);
    const float* d = D->dbuf + (size_t)s * D->slot_f_stride;
    float tau = (float)st.tau_pend;
    vbuf[outs[op] + i] = tau != 0.f ? u[i] - tau * d[i] : u[i];
  }
}

// Nodal fields at vbuf + offs[e] ([2][n][n], domain units) -> pixels dst + e * 2 * d_plane.
__global__ void __launch_bounds__(BLOCK) k_from_nodes_idx(const float* vbuf,
                                                          const long long* offs, int n,
                                                          float* dst, int H, long long d_plane,
                                                          int elems, float scale) {
  long long per = (long long)H * H;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < (long long)elems * 2 * per;
       k += (long long)gridDim.x * BLOCK) {
    int p = (int)(k / per);
    int e = p >> 1, comp = p & 1;
    int i = (int)(k % per);
    int a = i / H, b = i % H;
    dst[(size_t)e * 2 * d_plane + (size_t)comp * d_plane + i] =
        scale * vbuf[offs[e] + (size_t)comp * n * n + (size_t)a * n + b];
  }
}

// ------------------------------------------------------------------------------------------
// Rigid variant (definition of a rigid transformation): phi(x) = R(alpha) x + t with the three
// parameters in SlotState::rp, rotation about the domain origin as printed. A quadrature point
// q (in cells) maps to R(alpha) q + t / h. No field is stored: the energy passes and the
// gradient pass are reductions over the level's elements (the field energy pass's tiles). The energy
// is -NCC (no regulariser); the parameter gradient is
//   dE/dp_k = sum_q f_q grad T(phi(q)) . dphi/dp_k(q),   dphi/dalpha = R'(alpha) q, dphi/dt = I,
// f_q as in the gradient kernel; steepest descent in the parameters.

// The map in cells as a displacement, phi(q) - q = (R - I) q + t / h: positions are formed
// like the field kernels' (a node plus a small offset), so FP32 keeps them to ~1e-7 cells
// however far the point is from the rotation centre. Per element the node's offset is taken
// in FP64, per quadrature point the small (R - I)(xi, eta) is added in FP32.
struct RigidMap {
  double cm1, s, ox, oy;  // cos - 1 (as -2 sin^2(a/2)), sin, t / h (cells)
};
__device__ __forceinline__ RigidMap rigid_map(double a, double t0, double t1, int n) {
  RigidMap m;
  double sh = sin(0.5 * a);
  m.cm1 = -2.0 * sh * sh;
  m.s = sin(a);
  m.ox = t0 * (n - 1);
  m.oy = t1 * (n - 1);
  return m;
}
// offset (cells) of node (a, b) under the map
__device__ __forceinline__ void rigid_node_offset(const RigidMap& m, int a, int b, float& dx,
                                                  float& dy) {
  dx = (float)(m.cm1 * b - m.s * a + m.ox);
  dy = (float)(m.s * b + m.cm1 * a + m.oy);
}

// Energy of the rigid parameters (MODE 0: at rp for slots starting a level; MODE 1: at
// rp - tau_j rd for the NC steps of a line-search pass), one element tile. Partials as the
// field energy pass's, the three regulariser columns zero.
template <int MODE, int NC>
__device__ __forceinline__ void rigid_energy_item(BatchDesc* D, int s, int t, float* s_r,
                                                  double* s_stage) {
  constexpr int NXN = ET_X + 1, NYN = ET_Y + 1, NN = NXN * NYN;
  constexpr int NV = 3 * NC + 3;
  const int kind = MODE ? WK_LADDER : WK_EVAL;
  {
    const SlotState* stp = D->state + s;
    int ph = stp->phase;
    if (MODE == 0 && !(ph == PH_INIT || ph == PH_PROLONG)) return;
    if (MODE == 1 && ph != PH_LADDER) return;
    int l = (ph == PH_PROLONG) ? stp->level + 1 : stp->level;
    int n = lvl_n(l);
    const float* R = uni(D->pyr + D->frame_off[(size_t)stp->ref * PPRS_MAXL + l]);
    const float* TC = uni(D->tcoef + 4 * D->frame_off[(size_t)stp->tmpl * PPRS_MAXL + l]);
    const unsigned n16 = (unsigned)n << 4;
    double top = MODE ? stp->top : 0.0;
    RigidMap mp[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      double tj = MODE ? ldexp(top, -j) : 0.0;
      mp[j] = rigid_map(stp->rp[0] - tj * stp->rd[0], stp->rp[1] - tj * stp->rd[1],
                        stp->rp[2] - tj * stp->rd[2], n);
    }
    int ntx = (n - 1 + ET_X - 1) / ET_X;
    int e0x = (t % ntx) * ET_X, e0y = (t / ntx) * ET_Y;
    __syncthreads();
    {
      constexpr int SIT = (NN + BLOCK - 1) / BLOCK;
      float vr[SIT];
#pragma unroll
      for (int it = 0; it < SIT; ++it) {
        int k = threadIdx.x + it * BLOCK;
        int a = e0y + k / NXN, b = e0x + k % NXN;
        vr[it] = gld(R, (k < NN && a < n && b < n) ? (size_t)a * n + b : 0);
      }
#pragma unroll
      for (int it = 0; it < SIT; ++it) {
        int k = threadIdx.x + it * BLOCK;
        int a = e0y + k / NXN, b = e0x + k % NXN;
        if (k < NN) s_r[k] = (a < n && b < n) ? vr[it] : 0.f;
      }
    }
    __syncthreads();
    // per-thread FP32 sums over the thread's elements of the tile (at most
    // ET_X * ET_Y / BLOCK), converted to FP64 once per tile
    float es[3 * NC];
#pragma unroll
    for (int k = 0; k < 3 * NC; ++k) es[k] = 0.f;
    for (int e = threadIdx.x; e < ET_X * ET_Y; e += BLOCK) {
      int ey = e / ET_X, ex = e % ET_X;
      int a = e0y + ey, b = e0x + ex;
      if (a >= n - 1 || b >= n - 1) continue;
      int k00 = ey * NXN + ex;
      float rr[4] = {s_r[k00], s_r[k00 + 1], s_r[k00 + NXN], s_r[k00 + NXN + 1]};
      float ndx[NC], ndy[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) rigid_node_offset(mp[j], a, b, ndx[j], ndy[j]);
      // the element's cell in the clamp bounds and the byte offset of its first node's record
      const float lox = (float)(-b), hix = (float)(n - 1 - b);
      const float loy = (float)(-a), hiy = (float)(n - 1 - a);
      const unsigned base16 = (unsigned)mad24(a, n, b) << 4;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float xi = q ? kGP1 : kGP0, eta = p ? kGP1 : kGP0;
          float p0 = (1.f - xi) * (1.f - eta), p1 = xi * (1.f - eta), p2 = (1.f - xi) * eta, p3 = xi * eta;
          float rq = p0 * rr[0] + p1 * rr[1] + p2 * rr[2] + p3 * rr[3];
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            float cm1 = (float)mp[j].cm1, sn = (float)mp[j].s;
            float tx = xi + (ndx[j] + fmaf(cm1, xi, -sn * eta));
            float ty = eta + (ndy[j] + fmaf(sn, xi, cm1 * eta));
            float tv = sample_cells(TC, n16, base16, lox, hix, loy, hiy, tx, ty);
            es[3 * j + 0] += tv;
            es[3 * j + 1] = fmaf(tv, tv, es[3 * j + 1]);
            es[3 * j + 2] = fmaf(tv, rq, es[3 * j + 2]);
          }
        }
      }
    }
    double acc[NV];
    const double w = 0.25 / ((double)(n - 1) * (double)(n - 1));
#pragma unroll
    for (int k = 0; k < 3 * NC; ++k) acc[k] = w * (double)es[k];
#pragma unroll
    for (int k = 3 * NC; k < NV; ++k) acc[k] = 0.0;
    block_sum_store<NV>(acc, s_stage, slot_partial(D, s, kind, t));
  }
}

// The rigid energy passes of a step in one launch: the start energies of the slots that begin a
// level (the eval list) and the line-search passes (the ladder list), one item space made of
// the two lists in that order (disjoint slot sets, as for the fields' k_energy_step).
template <int NC>
__global__ void __launch_bounds__(BLOCK) k_rigid_energy_step(BatchDesc* D) {
  constexpr int NXN = ET_X + 1, NYN = ET_Y + 1, NN = NXN * NYN;
  constexpr int NV = 3 * NC + 3, KG = NV < BLOCK / 16 ? NV : BLOCK / 16;
  __shared__ float s_r[NN];
  __shared__ double s_stage[KG * (BLOCK / 2)];  // the partial sums' reduction stage
  __shared__ int s_pos;
  const int ne = D->lists[WK_EVAL].total, nl = D->lists[WK_LADDER].total;
  const int total = ne + nl;
  if (total <= 0) return;
  int chunk = (total + gridDim.x - 1) / gridDim.x;
  int b0 = blockIdx.x * chunk, b1 = min(b0 + chunk, total);
  ItemCursor c;
  if (b0 < ne && cursor_range(D, WK_EVAL, b0, min(b1, ne), c, &s_pos)) {
    for (; c.item < c.end; ++c.item) {
      int s, t;
      cursor_slot(D, WK_EVAL, c, s, t);
      rigid_energy_item<0, 1>(D, s, t, s_r, s_stage);
    }
  }
  if (b1 > ne && cursor_range(D, WK_LADDER, max(b0, ne) - ne, b1 - ne, c, &s_pos)) {
    for (; c.item < c.end; ++c.item) {
      int s, t;
      cursor_slot(D, WK_LADDER, c, s, t);
      rigid_energy_item<1, NC>(D, s, t, s_r, s_stage);
    }
  }
}

// Parameter gradient of the slots in GRAD: three FP64 partials per element tile.
__global__ void __launch_bounds__(BLOCK) k_rigid_grad(BatchDesc* D) {
  constexpr int NXN = ET_X + 1, NYN = ET_Y + 1, NN = NXN * NYN;
  __shared__ float s_r[NN];
  __shared__ double s_stage[3 * (BLOCK / 2)];  // the partial sums' reduction stage
  __shared__ int s_pos;
  ItemCursor c;
  if (!cursor_begin(D, WK_GRAD, c, &s_pos)) return;
  for (; c.item < c.end; ++c.item) {
    int s, t;
    cursor_slot(D, WK_GRAD, c, s, t);
    const SlotState* stp = D->state + s;
    if (stp->phase != PH_GRAD) continue;
    int l = stp->level;
    int n = lvl_n(l);
    const float* R = uni(D->pyr + D->frame_off[(size_t)stp->ref * PPRS_MAXL + l]);
    const float* T = uni(D->pyr + D->frame_off[(size_t)stp->tmpl * PPRS_MAXL + l]);
    RigidMap mp = rigid_map(stp->rp[0], stp->rp[1], stp->rp[2], n);
    const float cm1 = (float)mp.cm1, sn = (float)mp.s, cs = (float)cos(stp->rp[0]);
    double sg = stp->sigma;
    float inv_sig = sg > 0.0 ? (float)(1.0 / sg) : 0.f;
    float ncc = (float)stp->ncc, mean = (float)stp->mean;
    float inv_h = (float)(n - 1), h = 1.f / inv_h;
    float w = 0.25f / ((float)(n - 1) * (float)(n - 1));
    int ntx = (n - 1 + ET_X - 1) / ET_X;
    int e0x = (t % ntx) * ET_X, e0y = (t / ntx) * ET_Y;
    __syncthreads();
    {
      constexpr int SIT = (NN + BLOCK - 1) / BLOCK;
      float vr[SIT];
#pragma unroll
      for (int it = 0; it < SIT; ++it) {
        int k = threadIdx.x + it * BLOCK;
        int a = e0y + k / NXN, b = e0x + k % NXN;
        vr[it] = gld(R, (k < NN && a < n && b < n) ? (size_t)a * n + b : 0);
      }
#pragma unroll
      for (int it = 0; it < SIT; ++it) {
        int k = threadIdx.x + it * BLOCK;
        int a = e0y + k / NXN, b = e0x + k % NXN;
        if (k < NN) s_r[k] = (a < n && b < n) ? vr[it] : 0.f;
      }
    }
    __syncthreads();
    // per-thread FP32 sums over the thread's elements of the tile, converted to FP64 once
    float ga = 0.f, g0 = 0.f, g1 = 0.f;
    for (int e = threadIdx.x; e < ET_X * ET_Y; e += BLOCK) {
      int ey = e / ET_X, ex = e % ET_X;
      int a = e0y + ey, b = e0x + ex;
      if (a >= n - 1 || b >= n - 1) continue;
      int k00 = ey * NXN + ex;
      float rr[4] = {s_r[k00], s_r[k00 + 1], s_r[k00 + NXN], s_r[k00 + NXN + 1]};
      float ndx, ndy;
      rigid_node_offset(mp, a, b, ndx, ndy);
#pragma unroll
      for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float xi = q ? kGP1 : kGP0, eta = p ? kGP1 : kGP0;
          float p0 = (1.f - xi) * (1.f - eta), p1 = xi * (1.f - eta), p2 = (1.f - xi) * eta, p3 = xi * eta;
          float rq = p0 * rr[0] + p1 * rr[1] + p2 * rr[2] + p3 * rr[3];
          float tx = xi + (ndx + fmaf(cm1, xi, -sn * eta));
          float ty = eta + (ndy + fmaf(sn, xi, cm1 * eta));
          float gx, gy;
          float tv = sample_bil<true>(T, n, b, tx, a, ty, inv_h, &gx, &gy);
          float f = -w * (rq - ncc * (tv - mean) * inv_sig) * inv_sig;
          // dphi/dalpha = R'(alpha) q in domain units
          float qxd = ((float)b + xi) * h, qyd = ((float)a + eta) * h;
          float dax = -sn * qxd - cs * qyd, day = cs * qxd - sn * qyd;
          ga += f * (gx * dax + gy * day);
          g0 += f * gx;
          g1 += f * gy;
        }
      }
    }
    const double acc[3] = {(double)ga, (double)g0, (double)g1};
    block_sum_store<3>(acc, s_stage, slot_partial(D, s, WK_GRAD, t));
  }
}

// Per slot after the gradient pass: steepest-descent direction rd = grad, G.d = |grad|^2,
// max |d| over the level's nodes of the direction's displacement field (affine: its extreme
// at a corner of the domain), then the line-search start as for the fields.
__global__ void __launch_bounds__(BLOCK) k_rigid_grad_fin(BatchDesc* D) {
  __shared__ double s_red[(BLOCK / 64) * 3];
  const WorkList wl = D->lists[WK_GRAD];
  for (int pos = blockIdx.x; pos < wl.n_slots; pos += gridDim.x) {
    int s = D->list_slots[(size_t)WK_GRAD * D->max_slots + pos];
    SlotState* stp = D->state + s;
    if (stp->phase != PH_GRAD) continue;
    int l = stp->level;
    int n = lvl_n(l);
    double tot[3];
    sum_partials<3>(D, s, WK_GRAD, D->geom[l].tiles_elem, tot, s_red, false);
    if (threadIdx.x == 0) {
      SlotState st;
      load_head(st, *stp);
      D->node_count[(size_t)s * WK_COUNT + WK_GRAD] += (long long)n * n;
      double ca = cos(st.rp[0]), sa = sin(st.rp[0]);
      double dm = 0.0;
      for (int k = 0; k < 3; ++k) st.rd[k] = tot[k];
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          double dx = st.rd[0] * (-sa * cx - ca * cy) + st.rd[1];
          double dy = st.rd[0] * (ca * cx - sa * cy) + st.rd[2];
          dm = fmax(dm, fmax(fabs(dx), fabs(dy)));
        }
      st.gtd = tot[0] * tot[0] + tot[1] * tot[1] + tot[2] * tot[2];
      st.dmax = dm;
      if (!(st.gtd > 0.0) || !(st.dmax > 0.0)) {
        level_done(st);
      } else {
        double hh = 1.0 / (n - 1);
        st.tau_max = D->step_cap * hh / st.dmax;
        st.top = fmin(ldexp(st.tau_prev, D->ladder_k), st.tau_max);
        st.rung = 0;
        if (st.top < D->tau_min_rel * st.tau_max) level_done(st);
        else st.phase = PH_LADDER;
      }
      store_head(*stp, st);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// Series averaging: avg(x) = 1/N sum_i f_i(x + u_i(x)) over the aligned frames f_i o phi_{0,i}
// (pixel grid, bilinear, clamped to [0, W-1] x [0, H-1]). One pixel per lane; the frames are
// taken four at a time so a lane has 8 displacement loads and 16 frame loads in flight; the sum
// runs in FP64 in frame order, so every pixel's result is fixed whatever the launch.

__device__ __forceinline__ float sample_px(const float* f, int H, int W, float x, float y) {
  x = fminf(fmaxf(x, 0.f), (float)(W - 1));
  y = fminf(fmaxf(y, 0.f), (float)(H - 1));
  int x0 = min((int)floorf(x), W - 2), y0 = min((int)floorf(y), H - 2);
  float fx = x - (float)x0, fy = y - (float)y0;
  const GAS float* p = (const GAS float*)f + (size_t)y0 * W + x0;
  float v00 = p[0], v01 = p[1], v10 = p[W], v11 = p[W + 1];
  float top = fmaf(fx, v01 - v00, v00);
  float bot = fmaf(fx, v11 - v10, v10);
  return fmaf(fy, bot - top, top);
}

__global__ void __launch_bounds__(BLOCK) k_series_average(const float* frames, const float* u,
                                                          int N, int H, int W, float* out) {
  const long long plane = (long long)H * W;
  for (long long k = blockIdx.x * (long long)BLOCK + threadIdx.x; k < plane;
       k += (long long)gridDim.x * BLOCK) {
    int r = (int)(k / W), c = (int)(k - (long long)r * W);
    double acc = 0.0;
    int i = 0;
    for (; i + 4 <= N; i += 4) {
      float ux[4], uy[4], v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ux[q] = gld(u, (size_t)(i + q) * 2 * plane + k);
        uy[q] = gld(u, (size_t)(i + q) * 2 * plane + plane + k);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        v[q] = sample_px(frames + (size_t)(i + q) * plane, H, W, (float)c + ux[q], (float)r + uy[q]);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc += (double)v[q];
    }
    for (; i < N; ++i) {
      float ux = gld(u, (size_t)i * 2 * plane + k), uy = gld(u, (size_t)i * 2 * plane + plane + k);
      acc += (double)sample_px(frames + (size_t)i * plane, H, W, (float)c + ux, (float)r + uy);
    }
    gst(out, k, (float)(acc / N));
  }
}

// ------------------------------------------------------------------------------------------
// Host launch wrappers

namespace pprs_k {

static int grid_for(long long work, int cap = 8192) {
  long long g = (work + BLOCK - 1) / BLOCK;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t plan(BatchDesc* d, hipStream_t st) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(PLAN_T), 0, st, d);
  return hipGetLastError();
}
bool ladder_rungs_ok(int nc) { return nc == 1 || nc == 2 || nc == 3 || nc == 5 || nc == 7; }
hipError_t energy_step(BatchDesc* d, int nc, int grid, hipStream_t st) {
  switch (nc) {
    case 1: hipLaunchKernelGGL((k_energy_step<1>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 2: hipLaunchKernelGGL((k_energy_step<2>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 3: hipLaunchKernelGGL((k_energy_step<3>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 5: hipLaunchKernelGGL((k_energy_step<5>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 7: hipLaunchKernelGGL((k_energy_step<7>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t energy_step_fin(BatchDesc* d, int nc, int grid, hipStream_t st) {
  switch (nc) {
    case 1: hipLaunchKernelGGL((k_energy_step_fin<1>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 2: hipLaunchKernelGGL((k_energy_step_fin<2>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 3: hipLaunchKernelGGL((k_energy_step_fin<3>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 5: hipLaunchKernelGGL((k_energy_step_fin<5>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 7: hipLaunchKernelGGL((k_energy_step_fin<7>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t smooth_fin(BatchDesc* d, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_smooth_fin, dim3(grid), dim3(BLOCK), 0, st, d);
  return hipGetLastError();
}
const int kGradTiles[4][2] = {{32, 16}, {64, 8}, {128, 4}, {64, 16}};
void grad_tile(int variant, int* tx, int* ty) {
  if (variant < 0 || variant > 3) variant = 0;
  *tx = kGradTiles[variant][0];
  *ty = kGradTiles[variant][1];
}
hipError_t grad(BatchDesc* d, int variant, int grid, hipStream_t st) {
  switch (variant) {
    case 1: hipLaunchKernelGGL((k_grad<64, 8>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 2: hipLaunchKernelGGL((k_grad<128, 4>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 3: hipLaunchKernelGGL((k_grad<64, 16>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    default: hipLaunchKernelGGL((k_grad<32, 16>), dim3(grid), dim3(BLOCK), 0, st, d); break;
  }
  return hipGetLastError();
}
hipError_t smooth(BatchDesc* d, int dir, bool big, int grid, size_t lds_bytes, hipStream_t st) {
  if (big) {
    if (dir == 0) hipLaunchKernelGGL((k_smooth<0, true>), dim3(grid), dim3(SM_THREADS), lds_bytes, st, d);
    else hipLaunchKernelGGL((k_smooth<1, true>), dim3(grid), dim3(SM_THREADS), lds_bytes, st, d);
  } else {
    if (dir == 0) hipLaunchKernelGGL((k_smooth<0, false>), dim3(grid), dim3(SM_THREADS), lds_bytes, st, d);
    else hipLaunchKernelGGL((k_smooth<1, false>), dim3(grid), dim3(SM_THREADS), lds_bytes, st, d);
  }
  return hipGetLastError();
}
hipError_t smooth_win(BatchDesc* d, int halo, int grid, hipStream_t st) {
  if (halo == 16) hipLaunchKernelGGL(k_smooth_win<16>, dim3(grid), dim3(SW_THREADS), 0, st, d);
  else if (halo == 24) hipLaunchKernelGGL(k_smooth_win<24>, dim3(grid), dim3(SW_THREADS), 0, st, d);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t set_smooth_lds(size_t bytes) {
  const void* fns[4] = {(const void*)k_smooth<0, false>, (const void*)k_smooth<1, false>,
                        (const void*)k_smooth<0, true>, (const void*)k_smooth<1, true>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
hipError_t restrict_planes(const float* src, long long s_outer, long long s_inner, float* dst,
                           long long d_outer, long long d_inner, int inner, int nf, int planes,
                           hipStream_t st) {
  int nc = (nf - 1) / 2 + 1;
  hipLaunchKernelGGL(k_restrict, dim3(grid_for((long long)planes * nc * nc)), dim3(BLOCK), 0,
                     st, src, s_outer, s_inner, dst, d_outer, d_inner, inner, nf, planes);
  return hipGetLastError();
}
hipError_t to_nodes(const float* src, int H, long long s_plane, float* dst, int n,
                    long long d_plane, int planes, float scale, hipStream_t st) {
  hipLaunchKernelGGL(k_to_nodes, dim3(grid_for((long long)planes * n * n)), dim3(BLOCK), 0, st,
                     src, H, s_plane, dst, n, d_plane, planes, scale);
  return hipGetLastError();
}
hipError_t from_nodes(const float* src, int n, long long s_plane, float* dst, int H,
                      long long d_plane, int planes, float scale, hipStream_t st) {
  hipLaunchKernelGGL(k_from_nodes, dim3(grid_for((long long)planes * H * H)), dim3(BLOCK), 0,
                     st, src, n, s_plane, dst, H, d_plane, planes, scale);
  return hipGetLastError();
}
hipError_t tcoef(const float* f, int n, int N, float* coef, hipStream_t st) {
  long long total = (long long)N * n * n;
  long long g = (total + BLOCK - 1) / BLOCK;
  g = g < 1 ? 1 : (g > 16384 ? 16384 : g);
  hipLaunchKernelGGL(k_tcoef, dim3((unsigned)g), dim3(BLOCK), 0, st, f, n, total,
                     (float4*)coef);
  return hipGetLastError();
}
hipError_t fill(float* p, long long count, float v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(count)), dim3(BLOCK), 0, st, p, count, v);
  return hipGetLastError();
}
hipError_t fill_strided(float* p, long long outer, long long per, int n_outer, float v,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_fill_strided, dim3(grid_for((long long)n_outer * per)), dim3(BLOCK), 0,
                     st, p, outer, per, n_outer, v);
  return hipGetLastError();
}
hipError_t elem_sums(const float* src, long long plane_stride, int n, int bands, int planes,
                     double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_elem_sums, dim3(planes * bands), dim3(BLOCK), 0, st, src, plane_stride,
                     n, bands, partial);
  return hipGetLastError();
}
hipError_t elem_final(const double* partial, int bands, int planes, int mode, double* ms,
                      double* rsum, int rs_stride, int rs_off, hipStream_t st) {
  hipLaunchKernelGGL(k_elem_final, dim3((planes + 255) / 256), dim3(256), 0, st, partial, bands,
                     planes, mode, ms, rsum, rs_stride, rs_off);
  return hipGetLastError();
}
hipError_t normalize(float* f, long long plane_stride, long long per_plane, int planes,
                     const double* ms, hipStream_t st) {
  hipLaunchKernelGGL(k_normalize, dim3(grid_for((long long)planes * per_plane)), dim3(BLOCK), 0,
                     st, f, plane_stride, per_plane, planes, ms);
  return hipGetLastError();
}
hipError_t compose(const float* elems, long long estride, const int* left_idx,
                   const int* right_idx, float* out_base, long long ostride, int n, int ops,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_compose, dim3(grid_for((long long)ops * n * n)), dim3(BLOCK), 0, st,
                     elems, estride, left_idx, right_idx, out_base, ostride, n, ops);
  return hipGetLastError();
}
hipError_t finish(BatchDesc* d, const int* out_idx, float* elems, long long estride,
                  long long work, hipStream_t st) {
  hipLaunchKernelGGL(k_finish, dim3(grid_for(work)), dim3(BLOCK), 0, st, d, out_idx, elems,
                     estride);
  return hipGetLastError();
}

hipError_t pool_assign(BatchDesc* d, const SlotState* staged, const int* slots, int ops,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_pool_assign, dim3(grid_for((long long)ops * sizeof(SlotState) / 4)),
                     dim3(BLOCK), 0, st, d, staged, slots, ops);
  return hipGetLastError();
}
hipError_t pool_zero(BatchDesc* d, int l, int n_l, const int* slots, int ops, hipStream_t st) {
  hipLaunchKernelGGL(k_pool_zero, dim3(grid_for((long long)ops * 2 * n_l * n_l)), dim3(BLOCK), 0,
                     st, d, l, slots, ops);
  return hipGetLastError();
}
hipError_t pool_compose(BatchDesc* d, int L, const float* vbuf, const long long* off0,
                        const long long* off1, const int* slots, int ops, hipStream_t st) {
  long long n = (1LL << L) + 1;
  hipLaunchKernelGGL(k_pool_compose, dim3(grid_for((long long)ops * n * n)), dim3(BLOCK), 0, st,
                     d, L, vbuf, off0, off1, slots, ops);
  return hipGetLastError();
}
hipError_t pool_restrict(BatchDesc* d, int l, int n_c, const int* slots, int ops,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_pool_restrict, dim3(grid_for((long long)ops * 2 * n_c * n_c)),
                     dim3(BLOCK), 0, st, d, l, slots, ops);
  return hipGetLastError();
}
hipError_t pool_copy(BatchDesc* d, int l, int n_l, const float* src, long long sstride,
                     const int* src_idx, const int* slots, int ops, hipStream_t st) {
  hipLaunchKernelGGL(k_pool_copy, dim3(grid_for((long long)ops * 2 * n_l * n_l)), dim3(BLOCK), 0,
                     st, d, l, src, sstride, src_idx, slots, ops);
  return hipGetLastError();
}
hipError_t pool_copy_off(BatchDesc* d, int l, int n_l, const float* vbuf, const long long* offs,
                         const int* slots, int ops, hipStream_t st) {
  hipLaunchKernelGGL(k_pool_copy_off, dim3(grid_for((long long)ops * 2 * n_l * n_l)), dim3(BLOCK),
                     0, st, d, l, vbuf, offs, slots, ops);
  return hipGetLastError();
}
hipError_t pool_finish(BatchDesc* d, int L, const int* slots, const long long* outs, int ops,
                       float* vbuf, hipStream_t st) {
  long long n = (1LL << L) + 1;
  hipLaunchKernelGGL(k_pool_finish, dim3(grid_for((long long)ops * 2 * n * n)), dim3(BLOCK), 0,
                     st, d, L, slots, outs, ops, vbuf);
  return hipGetLastError();
}
hipError_t from_nodes_idx(const float* vbuf, const long long* offs, int n, float* dst, int H,
                          long long d_plane, int elems, float scale, hipStream_t st) {
  hipLaunchKernelGGL(k_from_nodes_idx, dim3(grid_for((long long)elems * 2 * H * H)), dim3(BLOCK),
                     0, st, vbuf, offs, n, dst, H, d_plane, elems, scale);
  return hipGetLastError();
}

hipError_t rigid_energy_step(BatchDesc* d, int nc, int grid, hipStream_t st) {
  switch (nc) {
    case 1: hipLaunchKernelGGL((k_rigid_energy_step<1>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 2: hipLaunchKernelGGL((k_rigid_energy_step<2>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 3: hipLaunchKernelGGL((k_rigid_energy_step<3>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 5: hipLaunchKernelGGL((k_rigid_energy_step<5>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    case 7: hipLaunchKernelGGL((k_rigid_energy_step<7>), dim3(grid), dim3(BLOCK), 0, st, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t rigid_grad(BatchDesc* d, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_rigid_grad, dim3(grid), dim3(BLOCK), 0, st, d);
  return hipGetLastError();
}
hipError_t rigid_grad_fin(BatchDesc* d, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_rigid_grad_fin, dim3(grid), dim3(BLOCK), 0, st, d);
  return hipGetLastError();
}

hipError_t series_average(const float* frames, const float* u, int N, int H, int W, float* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_series_average, dim3(grid_for((long long)H * W)), dim3(BLOCK), 0, st,
                     frames, u, N, H, W, out);
  return hipGetLastError();
}

}  // namespace pprs_k
