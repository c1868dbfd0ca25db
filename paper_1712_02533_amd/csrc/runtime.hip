// Host runtime and C-ABI of libpprs: context, device workspace, batched execution of
// registrations (one slot per A or B application), the series scan, and kernel timing.
//
// A batch runs as a sequence of identical "steps" (plan, prolong, eval, grad, smooth y,
// smooth x, line search). The device decides per slot what happens next; the host only
// launches steps and polls one counter of active slots between groups of steps, so slots
// retire independently and a batch mixes slots that are on different grid levels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>
#include <queue>
#include <functional>
#include <mutex>

#include "../../include/pprs.h"
#include "kernels.h"
#include "pprs_internal.h"

namespace pprs_cnn_api {
hipError_t pack_pairs(const float* lvl, int n, const int* ref, const int* tmpl, int P,
                      float* out, hipStream_t st);
pprs_status forward_into(pprs_cnn* c, const float* x, int B, float* y);
hipError_t planes_to_nhwc(const float* src, int n, long long pstride, int P, float scale,
                          float* out, hipStream_t st);
hipError_t nhwc_to_planes(const float* y, int S, int P, float scale, float* base,
                          long long stride, hipStream_t st);
int cnn_device(const pprs_cnn* c);
hipError_t check_pred(const float* y, int P, long long n_per, float limit, int* bad,
                      hipStream_t st);
}  // namespace pprs_cnn_api

static thread_local std::string g_err = "no error";

static pprs_status fail(pprs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(PPRS_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                  \
  } while (0)

#define STCHK(expr)                 \
  do {                              \
    pprs_status s_ = (expr);        \
    if (s_ < 0) return s_;          \
  } while (0)

namespace {

const int kGridFin = 512;       // finalisation: one workgroup per listed slot (grid-stride)
const int kPoolSlotsDefault = 512;  // concurrent registrations of a series (pprs_set_pool)

// A device buffer of a context: grown by ensure(), freed with the context unless it is a
// piece of the allocation-free entry point's scratch array (owned = false).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool owned = true;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p && owned) (void)hipFree(p);
  }
};

// The allocation-free entry point hands ensure() a bump arena over the device's scratch array
// for the duration of its call (set on the calling thread only): buffers are then carved from
// it instead of allocated.
struct Arena {
  char* base;
  size_t size, used;
  hipStream_t stream;
};
thread_local Arena* g_arena = nullptr;
const size_t kArenaAlign = 256;

enum { TK_PLAN = 0, TK_PROLONG, TK_EVAL, TK_GRAD, TK_SMY, TK_SMX, TK_LADDER, TK_FIN, TK_SMW,
       TK_COUNT };
const char* kTkName[TK_COUNT] = {"plan", "prolong", "energy_eval", "grad", "smooth_y",
                                 "smooth_x", "energy_ladder", "finalize", "smooth_window"};
// algorithmic HBM bytes per grid node (both displacement components) of one launch per kind
const double kBytesPerNode[TK_COUNT] = {0.0, 12.0, 16.0, 40.0, 16.0, 24.0, 24.0, 0.0, 16.0};

int level_n(int l) { return (1 << l) + 1; }

}  // namespace

struct pprs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // frames
  DevBuf frames, frame_off, rsum, fr_ms, fr_part, tcoef;
  std::vector<long long> frame_off_host;
  // slots
  DevBuf state, ubuf, dbuf, gbuf, zbuf, partial, nodecount, coef, list_slots, list_off,
      lists, desc, opidx;
  // scan elements [M][2][nL^2] and staging
  DevBuf elems;
  int* active_host = nullptr;
  bool log = false;  // one progress line per batch on stderr (environment PPRS_LOG=1)
  pprs_cnn* cnn = nullptr;  // warm start network (not owned)
  double warm_max_cells = 8.0;
  int warm_mode = PPRS_WARM_REFINE;
  unsigned warm_levels = ~0u;  // bit L set: series with side 2^L use the warm start
  DevBuf cnn_in, cnn_out, tmp, badflags, warm_stage;
  DevBuf avg_stage;  // the series average of the averaging procedure ([H][W])
  // slot pool: one poll's packed uploads (finish lists, staged slot states, init lists)
  DevBuf pool_pack;
  int pool_group = 16;   // steps between polls of the slot pool
  int pool_slots = kPoolSlotsDefault;  // concurrent registrations of a series
  // workgroups of the per-step item kernels (results do not depend on them)
  int grid_energy = 8192, grid_grad = 8192, grid_smooth = 8192, grid_prolong = 2048;
  bool smooth_window = false;  // windowed one-pass metric solve (opt-in, where beta allows)
  int tile_grad = 0;          // gradient tile setting (grad_variant maps it to the kernel's)
  int ladder_rungs = 0;       // step sizes per line-search pass (0: 2K+1)
  unsigned char* dlog = nullptr;  // decision log (caller's device buffer; pprs_set_decision_log)
  int dlog_cap = 0;
  long long dlog_row0 = 0;        // log row of the next batch's first registration
  int smooth_lines = 16;      // column-strip width of the line solves (8, 16 or 32)
  size_t lds_smooth[2] = {0, 0};
  BatchDesc hd;
  int slots_cap = 0, slots_L = -1, slots_m0 = -1;
  bool slots_fields = false;  // the per-slot field buffers (u, d, G, z) cover slots_cap slots
  double coef_beta = -1.0;
  int coef_L = -1, coef_m0 = -1;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev;   // pairs
  std::vector<int> ev_kind;
  double t_ms[TK_COUNT] = {0};
  long long t_launch[TK_COUNT] = {0};
  double t_bytes[TK_COUNT] = {0};
  long long nodes_acc[WK_COUNT] = {0};
  // every workspace buffer (for pprs_workspace_bytes; each frees itself with the context)
  std::vector<const DevBuf*> all_bufs() const {
    return {&frames, &frame_off, &rsum, &fr_ms, &fr_part, &tcoef, &state, &ubuf, &dbuf, &gbuf, &zbuf,
            &partial, &nodecount, &coef, &list_slots, &list_off, &lists, &desc, &opidx,
            &elems, &cnn_in, &cnn_out, &tmp, &badflags, &warm_stage, &avg_stage, &pool_pack};
  }
};

namespace {

pprs_status ensure(DevBuf& b, size_t bytes, bool zero = false) {
  if (b.bytes >= bytes && b.p) return PPRS_OK;
  if (g_arena) {
    size_t off = (g_arena->used + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    if (off + bytes > g_arena->size)
      return fail(PPRS_ENOMEM, "scratch array exhausted (%zu of %zu bytes needed)", off + bytes,
                  g_arena->size);
    b.p = g_arena->base + off;
    b.bytes = bytes;
    b.owned = false;
    g_arena->used = off + bytes;
    // the scratch keeps the previous call's contents: clear what must start at zero
    if (zero) HIPCHK(pprs_k::fill((float*)b.p, (long long)(bytes / sizeof(float)), 0.f,
                                  g_arena->stream));
    return PPRS_OK;
  }
  if (b.p) {
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (bytes == 0) return PPRS_OK;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(PPRS_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  if (zero) {
    e = hipMemset(b.p, 0, bytes);
    if (e != hipSuccess) return fail(PPRS_EHIP, "hipMemset failed: %s", hipGetErrorString(e));
  }
  return PPRS_OK;
}

template <class T>
T* P(DevBuf& b) {
  return reinterpret_cast<T*>(b.p);
}

pprs_status check_params(const pprs_params* p, int L) {
  if (!p) return fail(PPRS_EINVAL, "params is NULL");
  if (p->levels < 1 || p->levels > L || L - p->levels + 1 < 1)
    return fail(PPRS_EINVAL, "levels must be in [1, %d] for this frame size", L);
  if (!(p->lambda >= 0.0) || !(p->beta >= 0.0))
    return fail(PPRS_EINVAL, "lambda and beta must be >= 0");
  if (!(p->armijo_sigma > 0.0 && p->armijo_sigma < 1.0))
    return fail(PPRS_EINVAL, "armijo_sigma must be in (0, 1)");
  if (p->ladder_k < 0 || p->ladder_k > 3) return fail(PPRS_EINVAL, "ladder_k must be in [0, 3]");
  if (!(p->step_cap > 0.0)) return fail(PPRS_EINVAL, "step_cap must be > 0");
  if (!(p->tau_min_rel > 0.0 && p->tau_min_rel < 1.0))
    return fail(PPRS_EINVAL, "tau_min_rel must be in (0, 1)");
  if (!(p->eps >= 0.0)) return fail(PPRS_EINVAL, "eps must be >= 0");
  if (p->iter_max < 0) return fail(PPRS_EINVAL, "iter_max must be >= 0");
  if (p->scan < PPRS_SCAN_SEQUENTIAL || p->scan > PPRS_SCAN_REDUCE_THEN_SCAN)
    return fail(PPRS_EINVAL, "unknown scan kind %d", p->scan);
  if (p->scan_workers < 0)
    return fail(PPRS_EINVAL, "scan_workers must be >= 0 (got %d)", p->scan_workers);
  if ((p->warm_start != 0 && p->warm_start != 1) ||
      (p->force_fallback != 0 && p->force_fallback != 1))
    return fail(PPRS_EINVAL, "warm_start and force_fallback must be 0 or 1");
  return PPRS_OK;
}

// H is 2^L pixels or 2^L + 1 nodes; returns L or -1.
int frame_level(int H, int W) {
  if (H != W || H < 4) return -1;
  for (int L = 2; L <= 10; ++L)
    if (H == (1 << L) || H == (1 << L) + 1) return L;
  return -1;
}

void fill_geom(LevelGeom& g, int l, int coef_off) {
  int n = level_n(l);
  g.n = n;
  g.tiles_grad = 0;  // set per run from the gradient tile shape (set_grad_tiles)
  g.tiles_elem = ((n - 1 + ET_X - 1) / ET_X) * ((n - 1 + ET_Y - 1) / ET_Y);
  g.tiles_prol = ((n + PT_X - 1) / PT_X) * ((n + PT_Y - 1) / PT_Y);
  // column strips: set per run from the tuned width (set_run_geometry); 8 lines bound the
  // item count the partial records are sized for
  g.sm_lines = 8;
  g.sm_items = (n + 7) / 8;
  g.coef_off = coef_off;
  g.sw_tiles = std::max(1, (n - 1) / SW_T);
}

// Dynamic LDS of the line solves: dir 0 stages a strip of columns (n (lines + 1) floats),
// dir 1 the rows each wavefront solves.
size_t smooth_lds_bytes(const BatchDesc& hd, int dir) {
  size_t mx = 0;
  for (int l = hd.coarsest; l <= hd.finest; ++l) {
    const LevelGeom& g = hd.geom[l];
    size_t C = (g.n + 63) / 64;
    size_t Rw = C <= 9 ? 4 : 2;  // lines per wavefront (SmoothR in kernels.hip; at most 4)
    size_t a = (size_t)g.n * (g.sm_lines + 1), b = (BLOCK / 64) * Rw * (64 * C + 1);
    mx = std::max(mx, dir == 0 ? a : b);
  }
  return mx * sizeof(float);
}

// Gradient kernel variant of a tile_grad setting: 0 (default) = 64x8, 4 = 32x16; 1, 2 and 3
// are the kernel's own variants (64x8, 128x4, 64x16). 64x8 tiles take 30 KB of LDS (five
// workgroups per CU) against 53 KB for 64x16 (three), which outweighs their larger halo.
int grad_variant(int tile_grad) { return tile_grad == 0 ? 1 : tile_grad == 4 ? 0 : tile_grad; }

// Per-run geometry from the launch shape (before each batch is uploaded): gradient tiles of
// the chosen tile shape, column-strip width of the line solves (LDS permitting).
pprs_status set_grad_tiles(pprs_ctx* c) {
  int tx, ty;
  pprs_k::grad_tile(grad_variant(c->tile_grad), &tx, &ty);
  BatchDesc& hd = c->hd;
  for (int l = hd.coarsest; l <= hd.finest; ++l) {
    int n = level_n(l);
    LevelGeom& g = hd.geom[l];
    g.tiles_grad = std::max(1, (n - 1) / tx) * std::max(1, (n - 1) / ty);  // last tiles absorb node n-1
    int lines = c->smooth_lines;
    while (lines > 8 && (long long)n * (lines + 1) > SM_LDS_MAX_FLOATS) lines /= 2;
    g.sm_lines = lines;
    g.sm_items = (n + lines - 1) / lines;
  }
  size_t lds = std::max(smooth_lds_bytes(hd, 0), smooth_lds_bytes(hd, 1));
  if (lds > 65536) HIPCHK(pprs_k::set_smooth_lds(lds));
  return PPRS_OK;
}

// Halo of the windowed metric solve for beta: the LU recurrences of S1 = M1 + (beta h)^2 K1
// contract by rho per node, the smaller root of r^2 - q r + 1 with q = |diag / offdiag| =
// (2/3 + 2 beta^2) / |1/6 - beta^2| (h cancels). The smallest compiled halo H with
// rho^H <= 2^-24 (FP32 resolution) is used; 0 selects the exact two-pass line solves.
int window_halo(double beta) {
  double di = 2.0 / 3.0 + 2.0 * beta * beta, o = fabs(1.0 / 6.0 - beta * beta);
  double rho = 0.0;
  if (o > 0.0) {
    double q = di / o;
    rho = 0.5 * (q - sqrt(q * q - 4.0));
  }
  const double eps = ldexp(1.0, -24);
  for (int h : {16, 24})
    if (pow(rho, h) <= eps) return h;
  return 0;
}

// Bytes of the per-slot workspace for `cap` slots on levels m0..L (fields: the per-slot u, d,
// G and z buffers; the rigid variant has none).
struct SlotBytes {
  size_t state, ubuf, dbuf, gbuf, zbuf, partial, nodecount, coef, list_slots, list_off, lists,
      desc, opidx;
};

// Lays out the slot geometry of levels m0..L in hd (level geometry, u offsets, strides) and
// returns the buffer sizes for cap slots. ensure_slots allocates them; pprs_workspace_query
// adds them up.
SlotBytes slot_layout(BatchDesc& hd, int cap, int L, int m0, bool fields) {
  hd.finest = L;
  hd.coarsest = m0;
  int coef_off = 0;
  long long uoff = 0;
  int max_items = 1;
  for (int l = 0; l < PPRS_MAXL; ++l) hd.u_off[l] = 0;
  for (int l = m0; l <= L; ++l) {
    fill_geom(hd.geom[l], l, coef_off);
    coef_off += 3 * coef_pitch(hd.geom[l].n);
    hd.u_off[l] = uoff;
    uoff += 4LL * hd.geom[l].n * hd.geom[l].n;
    max_items = std::max(max_items, std::max(hd.geom[l].tiles_elem, 2 * hd.geom[l].sm_items));
    max_items = std::max(max_items, 2 * hd.geom[l].sw_tiles * hd.geom[l].sw_tiles);
  }
  int nL = level_n(L);
  hd.slot_u_stride = uoff;
  hd.slot_f_stride = 2LL * nL * nL;
  hd.slot_p_stride = 2LL * nL * row_pitch(nL);
  hd.part_kind_stride = (long long)max_items * PW;
  hd.part_slot_stride = hd.part_kind_stride * WK_COUNT;
  hd.max_slots = cap;
  SlotBytes b;
  b.state = sizeof(SlotState) * cap;
  b.ubuf = fields ? sizeof(float) * hd.slot_u_stride * cap : 0;
  b.dbuf = fields ? sizeof(float) * hd.slot_f_stride * cap : 0;
  b.gbuf = fields ? sizeof(float) * hd.slot_p_stride * cap : 0;
  b.zbuf = b.gbuf;
  b.partial = sizeof(double) * hd.part_slot_stride * cap;
  b.nodecount = sizeof(long long) * WK_COUNT * cap;
  b.coef = sizeof(float) * coef_off;
  b.list_slots = sizeof(int) * WK_COUNT * cap;
  b.list_off = sizeof(int) * WK_COUNT * (cap + 1);
  b.lists = sizeof(WorkList) * WK_COUNT;
  b.desc = sizeof(BatchDesc);
  b.opidx = sizeof(int) * 3 * cap;
  return b;
}

// Workspace for up to `cap` slots on levels m0..L, and the metric coefficients for beta.
// fields = false (the rigid variant): state, partials and lists only, no per-slot fields.
pprs_status ensure_slots(pprs_ctx* c, int cap, int L, int m0, double beta, bool fields = true) {
  BatchDesc& hd = c->hd;
  if (cap > c->slots_cap || L != c->slots_L || m0 != c->slots_m0 ||
      (fields && !c->slots_fields)) {
    cap = std::max(cap, c->slots_cap);
    SlotBytes b = slot_layout(hd, cap, L, m0, fields);
    STCHK(ensure(c->state, b.state));
    if (fields) {
      STCHK(ensure(c->ubuf, b.ubuf));
      STCHK(ensure(c->dbuf, b.dbuf, true));
      STCHK(ensure(c->gbuf, b.gbuf));
      STCHK(ensure(c->zbuf, b.zbuf));
    }
    STCHK(ensure(c->partial, b.partial));
    STCHK(ensure(c->nodecount, b.nodecount));
    STCHK(ensure(c->coef, b.coef));
    STCHK(ensure(c->list_slots, b.list_slots));
    STCHK(ensure(c->list_off, b.list_off));
    STCHK(ensure(c->lists, b.lists));
    STCHK(ensure(c->desc, b.desc));
    STCHK(ensure(c->opidx, b.opidx));
    hd.state = P<SlotState>(c->state);
    hd.ubuf = P<float>(c->ubuf);
    hd.dbuf = P<float>(c->dbuf);
    hd.gbuf = P<float>(c->gbuf);
    hd.zbuf = P<float>(c->zbuf);
    hd.partial = P<double>(c->partial);
    hd.node_count = P<long long>(c->nodecount);
    hd.coef = P<float>(c->coef);
    hd.list_slots = P<int>(c->list_slots);
    hd.list_off = P<int>(c->list_off);
    hd.lists = P<WorkList>(c->lists);
    hd.active_host = nullptr;  // the host polls the device word instead
    // the field buffers cover cap slots of this geometry only when allocated now
    c->slots_fields = fields;
    c->slots_cap = cap;
    c->slots_L = L;
    c->slots_m0 = m0;
    c->coef_beta = -1.0;
  }
  if (beta != c->coef_beta || c->coef_L != L || c->coef_m0 != m0) {
    // LU of S1 = M1 + (beta h)^2 K1 per level, in FP64, stored as FP32 a_i, 1/den_i, c'_i,
    // each array padded with zeros to coef_pitch(n) entries (the line solves read whole
    // lanes' chunks; zero coefficients make the padded nodes' maps constant zero).
    std::vector<float> host;
    for (int l = m0; l <= L; ++l) {
      int n = level_n(l);
      double h = 1.0 / (n - 1), cc = beta * beta * h * h;
      double de = h / 3.0 + cc / h, di = 2.0 * h / 3.0 + 2.0 * cc / h, o = h / 6.0 - cc / h;
      std::vector<double> den(n), cp(n);
      for (int i = 0; i < n; ++i) {
        double dd = (i == 0 || i == n - 1) ? de : di;
        den[i] = i == 0 ? dd : dd - o * cp[i - 1];
        cp[i] = o / den[i];
      }
      size_t base = host.size();
      const int cs = coef_pitch(n);
      host.resize(base + 3 * cs, 0.f);
      for (int i = 0; i < n; ++i) {
        host[base + i] = i == 0 ? 0.f : (float)(-o / den[i]);
        host[base + cs + i] = (float)(1.0 / den[i]);
        host[base + 2 * cs + i] = i == n - 1 ? 0.f : (float)cp[i];
      }
    }
    HIPCHK(hipMemcpy(c->coef.p, host.data(), host.size() * sizeof(float),
                     hipMemcpyHostToDevice));
    hd.smooth_halo = c->smooth_window ? window_halo(beta) : 0;
    c->coef_beta = beta;
    c->coef_L = L;
    c->coef_m0 = m0;
  }
  return PPRS_OK;
}

// One series' frames for prepare_series: device [N][H][H], levels m0..L, global index of its
// first frame f0. Frame f is checked for being constant when it serves as a reference:
// f < n_ref, or ref_mask[f] != 0 when a mask is given.
struct SeriesIn {
  const float* frames;
  int N, H, L, m0, f0, n_ref;
  const std::vector<char>* ref_mask;
};

const int kSumBands = 16;  // row bands of the per-frame sums (elem_sums)

// Buffer sizes of prepare_series for NT frames in all, at most Nmax per series, `nodes` grid
// nodes over all pyramids.
struct FrameBytes {
  size_t frames, frame_off, rsum, fr_part, fr_ms, tcoef;
};
FrameBytes frame_bytes(size_t nodes, int NT, int Nmax) {
  FrameBytes b;
  b.frames = sizeof(float) * std::max<size_t>(nodes, 1);
  b.tcoef = 4 * b.frames;  // bilinear coefficients of every node (template samples)
  b.frame_off = sizeof(long long) * (size_t)NT * PPRS_MAXL;
  b.rsum = sizeof(double) * (size_t)NT * PPRS_MAXL;
  b.fr_part = sizeof(double) * 2 * (size_t)Nmax * kSumBands;
  b.fr_ms = sizeof(double) * 2 * (size_t)Nmax * PPRS_MAXL;
  return b;
}

// Normalised frame pyramids of several series in one buffer: series s, level l is a block of
// N_s frames; the offset table maps (global frame, level) to the frame's first node.
pprs_status prepare_series(pprs_ctx* c, const std::vector<SeriesIn>& ser) {
  BatchDesc& hd = c->hd;
  int NT = 0, Nmax = 1;
  for (const SeriesIn& x : ser) {
    NT = std::max(NT, x.f0 + x.N);
    Nmax = std::max(Nmax, x.N);
  }
  std::vector<long long>& off = c->frame_off_host;
  off.assign((size_t)NT * PPRS_MAXL, -1);
  size_t total = 0;
  for (const SeriesIn& x : ser)
    for (int l = x.m0; l <= x.L; ++l) {
      size_t nn = (size_t)level_n(l) * level_n(l);
      for (int f = 0; f < x.N; ++f) off[(size_t)(x.f0 + f) * PPRS_MAXL + l] = total + f * nn;
      total += (size_t)x.N * nn;
    }
  FrameBytes fb = frame_bytes(total, NT, Nmax);
  STCHK(ensure(c->frames, fb.frames));
  STCHK(ensure(c->tcoef, fb.tcoef));
  STCHK(ensure(c->frame_off, fb.frame_off));
  STCHK(ensure(c->rsum, fb.rsum));
  const int bands = kSumBands;
  STCHK(ensure(c->fr_part, fb.fr_part));
  STCHK(ensure(c->fr_ms, fb.fr_ms));
  HIPCHK(hipMemcpyAsync(c->frame_off.p, off.data(), sizeof(long long) * off.size(),
                        hipMemcpyHostToDevice, c->stream));
  hd.pyr = P<float>(c->frames);
  hd.frame_off = P<long long>(c->frame_off);
  hd.rsum = P<double>(c->rsum);
  hd.tcoef = P<float>(c->tcoef);
  for (const SeriesIn& x : ser) {
    int N = x.N;
    auto lvl = [&](int l) { return hd.pyr + off[(size_t)x.f0 * PPRS_MAXL + l]; };
    int nL = level_n(x.L);
    HIPCHK(pprs_k::to_nodes(x.frames, x.H, (long long)x.H * x.H, lvl(x.L), nL,
                            (long long)nL * nL, N, 1.0f, c->stream));
    for (int l = x.L; l > x.m0; --l) {
      int nf = level_n(l), nc = level_n(l - 1);
      HIPCHK(pprs_k::restrict_planes(lvl(l), (long long)nf * nf, 0, lvl(l - 1),
                                     (long long)nc * nc, 0, 1, nf, N, c->stream));
    }
    std::vector<double> ms(2 * (size_t)N);
    double* rs = P<double>(c->rsum) + (size_t)x.f0 * PPRS_MAXL;
    for (int l = x.m0; l <= x.L; ++l) {
      int n = level_n(l);
      double* msd = P<double>(c->fr_ms) + 2 * (size_t)N * l;
      HIPCHK(pprs_k::elem_sums(lvl(l), (long long)n * n, n, bands, N, P<double>(c->fr_part),
                               c->stream));
      HIPCHK(pprs_k::elem_final(P<double>(c->fr_part), bands, N, 0, msd, nullptr, 0, 0,
                                c->stream));
      HIPCHK(hipMemcpyAsync(ms.data(), msd, sizeof(double) * 2 * N, hipMemcpyDeviceToHost,
                            c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      for (int f = 0; f < N; ++f) {
        double m = ms[2 * f], sg = ms[2 * f + 1];
        bool is_ref = x.ref_mask ? (*x.ref_mask)[f] != 0 : f < x.n_ref;
        if (sg <= 1e-12 * std::max(1.0, fabs(m)) && is_ref)
          return fail(PPRS_EINVAL, "reference frame %d is constant on level %d", f, l);
      }
      HIPCHK(pprs_k::normalize(lvl(l), (long long)n * n, (long long)n * n, N, msd, c->stream));
      HIPCHK(pprs_k::tcoef(lvl(l), n, N, hd.tcoef + 4 * off[(size_t)x.f0 * PPRS_MAXL + l],
                           c->stream));
      HIPCHK(pprs_k::elem_sums(lvl(l), (long long)n * n, n, bands, N, P<double>(c->fr_part),
                               c->stream));
      HIPCHK(pprs_k::elem_final(P<double>(c->fr_part), bands, N, 1, nullptr, rs, PPRS_MAXL, l,
                                c->stream));
    }
  }
  return PPRS_OK;
}

// Pyramids of one series of N frames (global frames 0 .. N-1).
pprs_status prepare_frames(pprs_ctx* c, const float* frames, int N, int H, int L, int m0,
                           int n_ref_frames, const std::vector<char>* ref_mask = nullptr) {
  std::vector<SeriesIn> one{SeriesIn{frames, N, H, L, m0, 0, n_ref_frames, ref_mask}};
  return prepare_series(c, one);
}

// First node of level l of global frame f (host-side pointer arithmetic on device memory).
float* frame_level_ptr(pprs_ctx* c, int f, int l) {
  return c->hd.pyr + c->frame_off_host[(size_t)f * PPRS_MAXL + l];
}

// ---- kernel timing -----------------------------------------------------------------------

pprs_status tk_begin(pprs_ctx* c, int kind, hipEvent_t* stop) {
  *stop = nullptr;
  if (!c->timing) return PPRS_OK;
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  HIPCHK(hipEventRecord(a, c->stream));
  c->ev.push_back(a);
  c->ev.push_back(b);
  c->ev_kind.push_back(kind);
  *stop = b;
  return PPRS_OK;
}
pprs_status tk_end(pprs_ctx* c, hipEvent_t stop) {
  if (stop) HIPCHK(hipEventRecord(stop, c->stream));
  return PPRS_OK;
}
pprs_status tk_collect(pprs_ctx* c) {
  for (size_t i = 0; i < c->ev_kind.size(); ++i) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
    c->t_ms[c->ev_kind[i]] += ms;
    c->t_launch[c->ev_kind[i]] += 1;
    (void)hipEventDestroy(c->ev[2 * i]);
    (void)hipEventDestroy(c->ev[2 * i + 1]);
  }
  c->ev.clear();
  c->ev_kind.clear();
  return PPRS_OK;
}

#define TIMED(kind, call)                 \
  do {                                    \
    hipEvent_t stop_;                     \
    STCHK(tk_begin(c, kind, &stop_));     \
    HIPCHK(call);                         \
    STCHK(tk_end(c, stop_));              \
  } while (0)

// Step sizes per line-search pass: the tuning value, else one group of 2K+1.
int ladder_rungs(const pprs_ctx* c, int K) { return c->ladder_rungs ? c->ladder_rungs : 2 * K + 1; }

// Upper bound on line-search passes per iteration (a guard against a run that never ends):
// groups of 2K+1 halvings from tau_max down to tau_min_rel tau_max, walked nc steps a pass.
long long ladder_pass_bound(const pprs_params* p, int nc) {
  int G = 2 * p->ladder_k + 1;
  long long groups = 2 + (long long)ceil(log2(1.0 / p->tau_min_rel) / G);
  return groups * G / nc + groups + 2;
}

// One step of every active slot: plan, gradient (with the prolongations of slots that
// finished a level), metric solve, line search.
pprs_status launch_step(pprs_ctx* c, BatchDesc* d, int nc) {
  size_t lds0 = c->lds_smooth[0], lds1 = c->lds_smooth[1];
  TIMED(TK_PLAN, pprs_k::plan(d, c->stream));
  TIMED(TK_GRAD, pprs_k::grad(d, grad_variant(c->tile_grad), c->grid_grad, c->stream));
  if (c->hd.smooth_halo) {
    TIMED(TK_SMW, pprs_k::smooth_win(d, c->hd.smooth_halo, c->grid_smooth, c->stream));
  } else {
    bool big = level_n(c->hd.finest) > 9 * 64;  // lines longer than 9 nodes per lane
    TIMED(TK_SMY, pprs_k::smooth(d, 0, big, c->grid_smooth, lds0, c->stream));
    TIMED(TK_SMX, pprs_k::smooth(d, 1, big, c->grid_smooth, lds1, c->stream));
  }
  TIMED(TK_FIN, pprs_k::smooth_fin(d, kGridFin, c->stream));
  // start energies of the slots that begin a level and the line-search passes, one launch
  TIMED(TK_LADDER, pprs_k::energy_step(d, nc, c->grid_energy, c->stream));
  TIMED(TK_FIN, pprs_k::energy_step_fin(d, nc, kGridFin, c->stream));
  return PPRS_OK;
}

// INIT_RESUME: the op continues, on its start level, a result another op left on the level
// below (copied in, then prolongated by the state machine as between two levels).
enum InitKind { INIT_IDENTITY = 0, INIT_COMPOSE = 1, INIT_GIVEN = 2, INIT_PREPARED = 3,
                INIT_RESUME = 4 };

// One step of the rigid variant: the parameter gradient with its finaliser, then in one launch
// the start energies of the slots that begin a level and the line-search passes (a slot that
// begins a level iterates from the next step on, as the plan lists it), and the finaliser the
// field path uses.
pprs_status launch_step_rigid(pprs_ctx* c, BatchDesc* d, int nc) {
  TIMED(TK_PLAN, pprs_k::plan(d, c->stream));
  TIMED(TK_GRAD, pprs_k::rigid_grad(d, c->grid_grad, c->stream));
  TIMED(TK_FIN, pprs_k::rigid_grad_fin(d, kGridFin, c->stream));
  // start energies of the slots that begin a level and the line-search passes, one launch
  TIMED(TK_LADDER, pprs_k::rigid_energy_step(d, nc, c->grid_energy, c->stream));
  TIMED(TK_FIN, pprs_k::energy_step_fin(d, nc, kGridFin, c->stream));
  return PPRS_OK;
}

// Runs n slots (reference ref[s], template tmpl[s]) to completion and writes each result
// (domain units, [2][nL][nL]) to elems[out_idx[s]]. INIT_COMPOSE composes elems[left[s]]
// and elems[right[s]]; INIT_GIVEN takes the finest-level guess already in slot 0's buffer.
pprs_status run_batch(pprs_ctx* c, int n, const int* ref, const int* tmpl, InitKind init,
                      const int* left, const int* right, const int* out_idx, float* elems,
                      const pprs_params* p, pprs_pair_stats* stats, long long* node_steps,
                      long long* node_passes, int* flags_or, int start = -1,
                      const int* start_level = nullptr, const int* extra_flags = nullptr) {
  if (n <= 0) return PPRS_OK;
  auto t_start = std::chrono::steady_clock::now();
  BatchDesc& hd = c->hd;
  int L = hd.finest, m0 = hd.coarsest;
  int nL = level_n(L);
  hd.n_slots = n;
  hd.ladder_k = p->ladder_k;
  hd.rigid = 0;
  hd.lambda = p->lambda;
  hd.sigma = p->armijo_sigma;
  hd.step_cap = p->step_cap;
  hd.tau_min_rel = p->tau_min_rel;
  hd.eps = p->eps;
  hd.iter_max = p->iter_max;
  STCHK(set_grad_tiles(c));
  BatchDesc* d = P<BatchDesc>(c->desc);
  hd.dlog = c->dlog ? c->dlog + (size_t)c->dlog_row0 * c->dlog_cap : nullptr;
  hd.dlog_cap = c->dlog_cap;
  HIPCHK(hipMemcpyAsync(d, &hd, sizeof(BatchDesc), hipMemcpyHostToDevice, c->stream));
  if (start < m0 || start > L) start = m0;
  std::vector<SlotState> st(n);
  for (int s = 0; s < n; ++s) {
    int lv = start_level ? start_level[s] : start;
    memset(&st[s], 0, sizeof(SlotState));
    st[s].phase = PH_INIT;
    st[s].level = lv;
    st[s].ref = ref[s];
    st[s].tmpl = tmpl[s];
    st[s].finest = L;
    st[s].coarsest = lv;
    st[s].tau_prev = INFINITY;
    st[s].op = s;
    st[s].flags = extra_flags ? extra_flags[s] : 0;
  }
  HIPCHK(hipMemcpyAsync(hd.state, st.data(), sizeof(SlotState) * n, hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipMemsetAsync(hd.node_count, 0, sizeof(long long) * WK_COUNT * n, c->stream));
  std::vector<int> idx(3 * (size_t)n);
  for (int s = 0; s < n; ++s) {
    idx[s] = left ? left[s] : 0;
    idx[n + s] = right ? right[s] : 0;
    idx[2 * n + s] = out_idx[s];
  }
  int* didx = P<int>(c->opidx);
  HIPCHK(hipMemcpyAsync(didx, idx.data(), sizeof(int) * 3 * n, hipMemcpyHostToDevice,
                        c->stream));
  long long est = 2LL * nL * nL;
  // initial guess on the start level (INIT_PREPARED: the caller filled it)
  if (init == INIT_IDENTITY) {
    int n0 = level_n(start);
    HIPCHK(pprs_k::fill_strided(hd.ubuf + hd.u_off[start], hd.slot_u_stride, 2LL * n0 * n0, n,
                                0.f, c->stream));
  } else if (init != INIT_PREPARED) {
    if (init == INIT_COMPOSE)
      HIPCHK(pprs_k::compose(elems, est, didx, didx + n, hd.ubuf + hd.u_off[L],
                             hd.slot_u_stride, nL, n, c->stream));
    for (int l = L; l > start; --l) {
      int nf = level_n(l), nc = level_n(l - 1);
      HIPCHK(pprs_k::restrict_planes(hd.ubuf + hd.u_off[l], hd.slot_u_stride, (long long)nf * nf,
                                     hd.ubuf + hd.u_off[l - 1], hd.slot_u_stride,
                                     (long long)nc * nc, 2, nf, 2 * n, c->stream));
    }
  }
  // steps
  c->lds_smooth[0] = smooth_lds_bytes(hd, 0);
  c->lds_smooth[1] = smooth_lds_bytes(hd, 1);
  int K = p->ladder_k, nc = ladder_rungs(c, K);
  long long passes_per_iter = ladder_pass_bound(p, nc);
  long long max_steps =
      (long long)p->levels * ((long long)p->iter_max + 2) * (passes_per_iter + 2) + 64;
  long long done_steps = 0;
  int group = 4;
  while (true) {
    for (int k = 0; k < group; ++k) STCHK(launch_step(c, d, nc));
    done_steps += group;
    int active = 0;
    HIPCHK(hipMemcpyAsync(&active, &d->active, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->timing) STCHK(tk_collect(c));
    if (active == 0) break;
    if (done_steps > max_steps)
      return fail(PPRS_ESTATE, "batch did not finish within %lld steps", max_steps);
    group = std::min(group * 2, 32);
  }
  HIPCHK(pprs_k::finish(d, didx + 2 * n, elems, est, (long long)n * est, c->stream));
  if (c->log) {
    HIPCHK(hipStreamSynchronize(c->stream));
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    fprintf(stderr, "[pprs] batch of %d registrations done after %lld steps, %.2f ms\n", n,
            done_steps, ms);
    fflush(stderr);
  }
  // statistics
  HIPCHK(hipMemcpyAsync(st.data(), hd.state, sizeof(SlotState) * n, hipMemcpyDeviceToHost,
                        c->stream));
  std::vector<long long> nodes((size_t)n * WK_COUNT);
  HIPCHK(hipMemcpyAsync(nodes.data(), hd.node_count, sizeof(long long) * WK_COUNT * n,
                        hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  float batch_ms = (float)std::chrono::duration<double, std::milli>(
                       std::chrono::steady_clock::now() - t_start).count();
  for (int s = 0; s < n; ++s) {
    if (flags_or) *flags_or |= st[s].flags;
    for (int k = 0; k < WK_COUNT; ++k) c->nodes_acc[k] += nodes[(size_t)s * WK_COUNT + k];
    for (int l = st[s].coarsest; l <= L; ++l) {
      long long nn = (long long)level_n(l) * level_n(l);
      if (node_steps) *node_steps += nn * st[s].iters[l - st[s].coarsest];
      if (node_passes) *node_passes += nn * st[s].passes[l - st[s].coarsest];
    }
    if (stats) {
      // indexed from the batch's coarsest level; levels a warm start skipped report 0
      pprs_pair_stats& o = stats[s];
      memset(&o, 0, sizeof o);
      for (int l = st[s].coarsest; l <= L; ++l) {
        o.iters[l - m0] = st[s].iters[l - st[s].coarsest];
        o.passes[l - m0] = st[s].passes[l - st[s].coarsest];
      }
      o.energy = st[s].E;
      o.ncc = st[s].ncc;
      o.flags = st[s].flags;
      o.ms = batch_ms;
    }
  }
  return PPRS_OK;
}

const int kWarmLevel = 7;     // the network works on 128^2 frames (level 7)
const int kWarmChunk = 64;    // pairs per network call
const int kPairChunk = 512;   // pairs per batch of pprs_register_pairs

// Network predictions for n pairs (ref[s], tmpl[s]) written as level-7 guesses (domain units,
// [2][129][129]) to dst + s * dst_stride; bad[s] = 1 for predictions that are not finite or
// exceed the bound (all of them when force_fallback is set).
pprs_status warm_predict(pprs_ctx* c, int f0, int n, const int* ref, const int* tmpl,
                         float* dst, long long dst_stride, std::vector<int>& bad,
                         bool force_fallback) {
  BatchDesc& hd = c->hd;
  int S = 1 << kWarmLevel;
  size_t per = (size_t)S * S * 2;
  int chunk = std::min(n, kWarmChunk);
  STCHK(ensure(c->cnn_in, sizeof(float) * per * chunk));
  STCHK(ensure(c->cnn_out, sizeof(float) * per * chunk));
  STCHK(ensure(c->badflags, sizeof(int) * 3 * (size_t)n));
  int* dref = P<int>(c->badflags);
  int* dtmpl = dref + n;
  int* dbad = dtmpl + n;
  HIPCHK(hipMemcpyAsync(dref, ref, sizeof(int) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(dtmpl, tmpl, sizeof(int) * n, hipMemcpyHostToDevice, c->stream));
  for (int p0 = 0; p0 < n; p0 += chunk) {
    int np = std::min(chunk, n - p0);
    HIPCHK(pprs_cnn_api::pack_pairs(frame_level_ptr(c, f0, kWarmLevel), S + 1, dref + p0,
                                    dtmpl + p0, np,
                                    P<float>(c->cnn_in), c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    STCHK(pprs_cnn_api::forward_into(c->cnn, P<float>(c->cnn_in), np, P<float>(c->cnn_out)));
    HIPCHK(pprs_cnn_api::check_pred(P<float>(c->cnn_out), np, (long long)per,
                                    (float)c->warm_max_cells, dbad + p0, c->stream));
    HIPCHK(pprs_cnn_api::nhwc_to_planes(P<float>(c->cnn_out), S, np, 1.0f / S,
                                        dst + (size_t)p0 * dst_stride, dst_stride, c->stream));
  }
  bad.assign(n, 0);
  HIPCHK(hipMemcpyAsync(bad.data(), dbad, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (force_fallback) bad.assign(n, 1);
  return PPRS_OK;
}

// Initial guesses of n slots (pairs ref[s], tmpl[s]) from the network. PPRS_WARM_REFINE:
// the level-7 prediction is restricted to the coarsest level m0 and every level runs;
// PPRS_WARM_SKIP: the prediction is the start on level 7 and the coarser levels are skipped.
// A rejected prediction starts from the identity on m0 and is flagged PPRS_FLAG_FALLBACK.
// lv[s] and fl[s] receive each slot's start level and flags for run_batch (INIT_PREPARED).
pprs_status warm_init(pprs_ctx* c, int n, const int* ref, const int* tmpl, int m0,
                      bool force_fallback, std::vector<int>& lv, std::vector<int>& fl) {
  BatchDesc& hd = c->hd;
  std::vector<int> bad;
  STCHK(warm_predict(c, 0, n, ref, tmpl, hd.ubuf + hd.u_off[kWarmLevel], hd.slot_u_stride,
                     bad, force_fallback));
  int n0 = level_n(m0);
  long long per0 = 2LL * n0 * n0;
  lv.assign(n, m0);
  fl.assign(n, 0);
  if (c->warm_mode == PPRS_WARM_SKIP) {
    HIPCHK(pprs_k::fill_strided(hd.ubuf + hd.u_off[m0], hd.slot_u_stride, per0, n, 0.f,
                                c->stream));
    for (int s = 0; s < n; ++s) lv[s] = bad[s] ? m0 : kWarmLevel;
  } else {
    for (int l = kWarmLevel; l > m0; --l) {
      int nf = level_n(l), nc = level_n(l - 1);
      HIPCHK(pprs_k::restrict_planes(hd.ubuf + hd.u_off[l], hd.slot_u_stride, (long long)nf * nf,
                                     hd.ubuf + hd.u_off[l - 1], hd.slot_u_stride,
                                     (long long)nc * nc, 2, nf, 2 * n, c->stream));
    }
    for (int s = 0; s < n; ++s)
      if (bad[s])
        HIPCHK(pprs_k::fill_strided(hd.ubuf + hd.u_off[m0] + (size_t)s * hd.slot_u_stride,
                                    hd.slot_u_stride, per0, 1, 0.f, c->stream));
  }
  for (int s = 0; s < n; ++s) fl[s] = bad[s] ? PPRS_FLAG_FALLBACK : 0;
  return PPRS_OK;
}

// ---- slot pool ---------------------------------------------------------------------------
// A registration ("op") reads frames ref/tmpl, starts from the identity, a composition of two
// finished results or a staged guess, and writes its finest-level result (nodal, domain units)
// to its own version buffer vbuf + ver_off[out]. Ops become ready when the ops producing their
// inputs have finished; ready ops are started in free slots in op order, and the slots keep
// stepping (early retirement: a finished slot takes the next ready op at the following poll).
// Ops of different series may have different finest levels L (slots are sized for the
// largest).

// The warm start's judge (CHOOSE_A: the warm registration stopped on level 7 against the
// identity's NCC there; CHOOSE_B: the composition against the network's guess by their energy on
// level 7) is resolved when the op starts, from the results of its two probes.
enum { CHOOSE_NONE = 0, CHOOSE_A = 1, CHOOSE_B = 2 };

struct PoolOp {
  int ref, tmpl;   // global frame indices
  InitKind init;   // INIT_IDENTITY, INIT_COMPOSE, INIT_PREPARED (staged guess) or INIT_RESUME
  int in0, in1;    // INIT_COMPOSE: versions composed (in1 o in0); INIT_RESUME: in0 resumed
  int out;         // version written
  int start;       // start level
  int flags;       // initial flags (e.g. PPRS_FLAG_FALLBACK)
  int stage;       // INIT_PREPARED: index of the staged guess
  int L, m0;       // finest level of the op's frames; its series' coarsest level (statistics)
  int stop = -1;   // level the op ends on and writes its version at (-1: L)
  int eval_only = 0;             // probe: the start energy only
  int choose = CHOOSE_NONE;      // judge resolved at start from probe0 and probe1 (op indices)
  int probe0 = -1, probe1 = -1;
  int stage_alt = -1;            // CHOOSE_B: staged network guess of the op's pair
  int stop_level() const { return stop < 0 ? L : stop; }
};

struct PoolSpec {
  const float* stage = nullptr;   // staged guesses [count][2][n^2] on stage_level
  long long stage_stride = 0;
  int stage_level = -1;
};

struct GraphExec {
  hipGraphExec_t exec = nullptr;
  ~GraphExec() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

// Bytes of one poll's packed upload for a pool of S slots: at most S finished slots (slot and
// version offset each), S starting registrations (staged state and slot) and their initial-
// guess lists (slot, stage index, two version offsets), every list 8-byte aligned, with one
// list per finest level and one per kind, finest and start level at most.
size_t pool_pack_bytes(int S) {
  const size_t lists = PPRS_MAXL + 2 + 4 * PPRS_MAXL * PPRS_MAXL;
  return (size_t)S * (sizeof(int) + sizeof(long long)) +
         (size_t)S * (sizeof(SlotState) + sizeof(int)) +
         (size_t)S * (2 * sizeof(int) + 2 * sizeof(long long)) + lists * 4 * 8;
}

pprs_status run_pool(pprs_ctx* c, std::vector<PoolOp>& ops, int S, float* vbuf,
                     const std::vector<long long>& ver_off, const pprs_params* p,
                     const PoolSpec& spec, pprs_pair_stats* stats, long long* node_steps,
                     long long* node_passes, int* flags_or,
                     std::vector<double>* finish_ms = nullptr) {
  const int n_ops = (int)ops.size();
  if (n_ops == 0) return PPRS_OK;
  auto t_start = std::chrono::steady_clock::now();
  BatchDesc& hd = c->hd;
  int Lmax = hd.finest, m0min = hd.coarsest;
  S = std::max(1, std::min(S, std::min(n_ops, hd.max_slots)));
  hd.n_slots = S;
  hd.ladder_k = p->ladder_k;
  hd.rigid = 0;
  hd.lambda = p->lambda;
  hd.sigma = p->armijo_sigma;
  hd.step_cap = p->step_cap;
  hd.tau_min_rel = p->tau_min_rel;
  hd.eps = p->eps;
  hd.iter_max = p->iter_max;
  STCHK(set_grad_tiles(c));
  BatchDesc* d = P<BatchDesc>(c->desc);
  hd.dlog = c->dlog ? c->dlog + (size_t)c->dlog_row0 * c->dlog_cap : nullptr;
  hd.dlog_cap = c->dlog_cap;
  HIPCHK(hipMemcpyAsync(d, &hd, sizeof(BatchDesc), hipMemcpyHostToDevice, c->stream));
  for (const PoolOp& o : ops)
    if (o.L > Lmax || o.start < m0min || o.start > o.stop_level() || o.stop_level() > o.L ||
        o.m0 > o.start || o.out < 0 || o.out >= (int)ver_off.size() ||
        (o.choose == CHOOSE_A && (o.probe0 < 0 || ops[o.probe0].stop_level() + 1 > o.L)))
      return fail(PPRS_ESTATE, "pool op outside the slot geometry");
  // dependencies: producers are the ops whose out is read
  std::vector<int> producer(ver_off.size(), -1);
  for (int i = 0; i < n_ops; ++i) producer[ops[i].out] = i;
  std::vector<int> remaining(n_ops, 0);
  std::vector<std::vector<int>> dependents(n_ops);
  for (int i = 0; i < n_ops; ++i) {
    std::vector<int> deps;
    if (ops[i].init == INIT_COMPOSE)
      for (int v : {ops[i].in0, ops[i].in1}) {
        int q = v >= 0 && v < (int)producer.size() ? producer[v] : -1;
        if (q < 0 || q >= i)
          return fail(PPRS_EINDEX, "op %d reads a version no earlier op writes", i);
        deps.push_back(q);
      }
    if (ops[i].choose != CHOOSE_NONE)  // the probes (CHOOSE_A resumes probe0's version)
      for (int q : {ops[i].probe0, ops[i].probe1}) {
        if (q < 0 || q >= i) return fail(PPRS_EINDEX, "op %d judges by a later op", i);
        deps.push_back(q);
      }
    std::sort(deps.begin(), deps.end());
    deps.erase(std::unique(deps.begin(), deps.end()), deps.end());
    for (int q : deps) {
      remaining[i]++;
      dependents[q].push_back(i);
    }
  }
  if (!stats) return fail(PPRS_ESTATE, "the slot pool needs per-op statistics");
  std::priority_queue<int, std::vector<int>, std::greater<int>> ready;
  for (int i = 0; i < n_ops; ++i)
    if (remaining[i] == 0) ready.push(i);
  // empty slots
  std::vector<SlotState> st(S);
  for (int s = 0; s < S; ++s) {
    memset(&st[s], 0, sizeof(SlotState));
    st[s].phase = PH_DONE;
    st[s].level = m0min;
  }
  HIPCHK(hipMemcpyAsync(hd.state, st.data(), sizeof(SlotState) * S, hipMemcpyHostToDevice,
                        c->stream));
  // Every poll uploads what it hands the device (the finished slots' result lists, the staged
  // states of the starting registrations and the index lists of their initial guesses) as one
  // packed buffer in one copy; the kernels read their lists from it in stream order, so a poll
  // waits for the device once (the state read-back).
  const size_t pack_cap = pool_pack_bytes(S);
  STCHK(ensure(c->pool_pack, pack_cap));
  char* dpack = P<char>(c->pool_pack);
  std::vector<char> hpack(pack_cap);
  size_t pack_used = 0;
  bool pack_over = false;
  auto put = [&](const void* src, size_t bytes) -> size_t {
    size_t o = (pack_used + 7) & ~(size_t)7;
    if (o + bytes > pack_cap) {
      pack_over = true;
      return 0;
    }
    memcpy(hpack.data() + o, src, bytes);
    pack_used = o + bytes;
    return o;
  };
  struct FinishList {
    int L, cnt;
    size_t slots, outs;
  };
  std::vector<FinishList> finish_lists;
  std::vector<int> slot_op(S, -1), free_slots;
  std::vector<double> op_start(n_ops, 0.0);
  for (int s = S - 1; s >= 0; --s) free_slots.push_back(s);
  std::vector<long long> nodes((size_t)S * WK_COUNT);
  c->lds_smooth[0] = smooth_lds_bytes(hd, 0);
  c->lds_smooth[1] = smooth_lds_bytes(hd, 1);
  int K = p->ladder_k, nc = ladder_rungs(c, K);
  long long passes_per_iter = ladder_pass_bound(p, nc);
  long long per_op_steps =
      (long long)(Lmax - m0min + 1) * ((long long)p->iter_max + 2) * (passes_per_iter + 2) + 64;
  long long max_steps = per_op_steps * (long long)(n_ops / S + 2) + 64;
  long long done_steps = 0;
  int done_ops = 0;
  std::vector<int> lst(S), lst_stage(S);
  std::vector<long long> lst_o0(S), lst_o1(S);
  std::vector<SlotState> h_states(S);
  int G = std::max(1, c->pool_group);
  // the G steps between polls always launch the same kernels with the same arguments (all
  // per-slot state lives on the device): one captured graph replays them, unless per-launch
  // timing events are wanted
  GraphExec graph;
  if (!c->timing) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    pprs_status cs = PPRS_OK;
    for (int k = 0; k < G && cs == PPRS_OK; ++k) cs = launch_step(c, d, nc);
    hipError_t ce = hipStreamEndCapture(c->stream, &g);
    if (cs != PPRS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return cs;
    }
    if (ce != hipSuccess) return fail(PPRS_EHIP, "graph capture failed: %s", hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(&graph.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess)
      return fail(PPRS_EHIP, "graph instantiation failed: %s", hipGetErrorString(ie));
  }
  // The finished slots' results go to their versions (grouped by finest level) before the
  // slots are handed to new registrations: those lists open the next upload.
  auto launch_finish = [&]() -> pprs_status {
    for (const FinishList& f : finish_lists)
      HIPCHK(pprs_k::pool_finish(d, f.L, (const int*)(dpack + f.slots),
                                 (const long long*)(dpack + f.outs), f.cnt, vbuf, c->stream));
    finish_lists.clear();
    return PPRS_OK;
  };
  while (done_ops < n_ops) {
    // 1. start ready ops in free slots (the upload already holds the last poll's finish lists)
    int na = 0;
    std::vector<int> a_slot, a_op;
    while (!free_slots.empty() && !ready.empty()) {
      int i = ready.top();
      ready.pop();
      int s = free_slots.back();
      free_slots.pop_back();
      slot_op[s] = i;
      op_start[i] = std::chrono::duration<double, std::milli>(
                        std::chrono::steady_clock::now() - t_start).count();
      a_slot.push_back(s);
      a_op.push_back(i);
      PoolOp& o = ops[i];
      if (o.choose == CHOOSE_A) {
        // the warm result on level 7 against the identity's NCC there (the probes' results)
        const pprs_pair_stats& w = stats[o.probe0];
        if (w.ncc >= stats[o.probe1].ncc && !(w.flags & PPRS_FLAG_NAN)) {
          o.init = INIT_RESUME;
          o.start = ops[o.probe0].stop_level() + 1;
        } else {
          o.init = INIT_IDENTITY;
          o.start = o.m0;
          o.flags |= PPRS_FLAG_FALLBACK;
        }
      } else if (o.choose == CHOOSE_B) {
        // the start with the lower energy on level 7: composition (probe0) or network (probe1)
        const pprs_pair_stats& q = stats[o.probe1];
        if (q.energy < stats[o.probe0].energy && !(q.flags & PPRS_FLAG_NAN)) {
          o.init = INIT_PREPARED;
          o.stage = o.stage_alt;
          o.flags |= PPRS_FLAG_NET_START;
        }
      }
      SlotState& x = h_states[na];
      memset(&x, 0, sizeof(SlotState));
      x.phase = PH_INIT;
      x.level = o.start;
      x.ref = o.ref;
      x.tmpl = o.tmpl;
      x.finest = o.stop_level();
      x.coarsest = o.start;
      x.tau_prev = INFINITY;
      x.op = i;
      x.flags = o.flags;
      x.eval_only = o.eval_only;
      if (o.init == INIT_RESUME) {
        // continues a level-(start - 1) result, prolongated to the start level by the state
        // machine (no pending step), which then takes its start energy there
        x.phase = PH_PROLONG;
        x.level = o.start - 1;
      }
      ++na;
    }
    // initial-guess lists per kind, finest level and start level
    struct InitList {
      int kind, Lv, lv, cnt;
      size_t slots, stage, o0, o1;
    };
    std::vector<InitList> init_lists;
    size_t a_states = 0, a_slots = 0;
    if (na > 0) {
      a_states = put(h_states.data(), sizeof(SlotState) * na);
      a_slots = put(a_slot.data(), sizeof(int) * na);
      for (int kind : {(int)INIT_IDENTITY, (int)INIT_COMPOSE, (int)INIT_PREPARED,
                       (int)INIT_RESUME}) {
        for (int Lv = m0min; Lv <= Lmax; ++Lv) {
          for (int lv = m0min; lv <= Lv; ++lv) {
            int cnt = 0;
            for (int k = 0; k < na; ++k) {
              const PoolOp& o = ops[a_op[k]];
              if ((int)o.init != kind || o.start != lv || o.L != Lv) continue;
              lst[cnt] = a_slot[k];
              lst_stage[cnt] = o.stage;
              lst_o0[cnt] = kind == INIT_COMPOSE || kind == INIT_RESUME ? ver_off[o.in0] : 0;
              lst_o1[cnt] = kind == INIT_COMPOSE ? ver_off[o.in1] : 0;
              ++cnt;
            }
            if (cnt == 0) continue;
            if (kind == INIT_PREPARED &&
                (!spec.stage || spec.stage_level < lv || spec.stage_level > Lv))
              return fail(PPRS_ESTATE, "staged guesses on level %d cannot start level %d",
                          spec.stage_level, lv);
            InitList il{kind, Lv, lv, cnt, 0, 0, 0, 0};
            il.slots = put(lst.data(), sizeof(int) * cnt);
            if (kind == INIT_PREPARED) il.stage = put(lst_stage.data(), sizeof(int) * cnt);
            if (kind == INIT_COMPOSE || kind == INIT_RESUME)
              il.o0 = put(lst_o0.data(), sizeof(long long) * cnt);
            if (kind == INIT_COMPOSE) il.o1 = put(lst_o1.data(), sizeof(long long) * cnt);
            init_lists.push_back(il);
          }
        }
      }
    }
    if (pack_over) return fail(PPRS_ESTATE, "pool upload exceeds its %zu bytes", pack_cap);
    if (pack_used > 0)
      HIPCHK(hipMemcpyAsync(dpack, hpack.data(), pack_used, hipMemcpyHostToDevice, c->stream));
    pack_used = 0;
    STCHK(launch_finish());
    if (na > 0) {
      HIPCHK(pprs_k::pool_assign(d, (const SlotState*)(dpack + a_states),
                                 (const int*)(dpack + a_slots), na, c->stream));
      for (const InitList& il : init_lists) {
        const int* ds = (const int*)(dpack + il.slots);
        const int lv = il.lv, Lv = il.Lv, cnt = il.cnt;
        int top = Lv;
        if (il.kind == INIT_IDENTITY) {
          HIPCHK(pprs_k::pool_zero(d, lv, level_n(lv), ds, cnt, c->stream));
          top = lv;
        } else if (il.kind == INIT_COMPOSE) {
          HIPCHK(pprs_k::pool_compose(d, Lv, vbuf, (const long long*)(dpack + il.o0),
                                      (const long long*)(dpack + il.o1), ds, cnt, c->stream));
        } else if (il.kind == INIT_RESUME) {
          // the resumed result into the first buffer of the level below the start
          HIPCHK(pprs_k::pool_copy_off(d, lv - 1, level_n(lv - 1), vbuf,
                                       (const long long*)(dpack + il.o0), ds, cnt, c->stream));
          top = lv;
        } else {
          HIPCHK(pprs_k::pool_copy(d, spec.stage_level, level_n(spec.stage_level), spec.stage,
                                   spec.stage_stride, (const int*)(dpack + il.stage), ds, cnt,
                                   c->stream));
          top = spec.stage_level;
        }
        for (int l = top; l > lv; --l)
          HIPCHK(pprs_k::pool_restrict(d, l, level_n(l - 1), ds, cnt, c->stream));
      }
    }
    // 2. step every slot G times
    if (graph.exec) {
      HIPCHK(hipGraphLaunch(graph.exec, c->stream));
    } else {
      for (int k = 0; k < G; ++k) STCHK(launch_step(c, d, nc));
    }
    done_steps += G;
    // 3. poll: retire finished slots, release their dependents
    HIPCHK(hipMemcpyAsync(st.data(), hd.state, sizeof(SlotState) * S, hipMemcpyDeviceToHost,
                          c->stream));
    // the per-kind node counts feed the kernel timing figures only
    if (c->timing)
      HIPCHK(hipMemcpyAsync(nodes.data(), hd.node_count, sizeof(long long) * WK_COUNT * S,
                            hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->timing) STCHK(tk_collect(c));
    std::vector<int> fin;
    for (int s = 0; s < S; ++s) {
      int i = slot_op[s];
      if (i < 0 || st[s].phase != PH_DONE) continue;
      fin.push_back(s);
      const PoolOp& op = ops[i];
      // a probe's non-finite energy only decides its judge; it does not fail the call
      bool probe = op.eval_only || op.stop_level() < op.L;
      if (flags_or) *flags_or |= probe ? (st[s].flags & ~PPRS_FLAG_NAN) : st[s].flags;
      if (c->timing)
        for (int k = 0; k < WK_COUNT; ++k) c->nodes_acc[k] += nodes[(size_t)s * WK_COUNT + k];
      for (int l = st[s].coarsest; l <= op.stop_level(); ++l) {
        long long nn = (long long)level_n(l) * level_n(l);
        if (node_steps) *node_steps += nn * st[s].iters[l - st[s].coarsest];
        if (node_passes) *node_passes += nn * st[s].passes[l - st[s].coarsest];
      }
      if (stats) {
        pprs_pair_stats& o = stats[i];
        memset(&o, 0, sizeof o);
        for (int l = st[s].coarsest; l <= op.stop_level(); ++l) {
          o.iters[l - op.m0] = st[s].iters[l - st[s].coarsest];
          o.passes[l - op.m0] = st[s].passes[l - st[s].coarsest];
        }
        o.energy = st[s].E;
        o.ncc = st[s].ncc;
        o.flags = st[s].flags;
      }
      double now_ms = std::chrono::duration<double, std::milli>(
                          std::chrono::steady_clock::now() - t_start).count();
      if (stats) stats[i].ms = (float)(now_ms - op_start[i]);
      if (finish_ms) (*finish_ms)[i] = now_ms;
      for (int q : dependents[i])
        if (--remaining[q] == 0) ready.push(q);
      ++done_ops;
    }
    // the finished results' lists (grouped by finest level) open the next upload; their slots
    // are free for the registrations that upload starts (pool_finish runs before pool_assign)
    for (int Lv = m0min; Lv <= Lmax && !fin.empty(); ++Lv) {
      int cnt = 0;
      for (int s : fin)
        if (ops[slot_op[s]].stop_level() == Lv) {
          lst[cnt] = s;
          lst_o0[cnt] = ver_off[ops[slot_op[s]].out];
          ++cnt;
        }
      if (cnt == 0) continue;
      FinishList f{Lv, cnt, 0, 0};
      f.slots = put(lst.data(), sizeof(int) * cnt);
      f.outs = put(lst_o0.data(), sizeof(long long) * cnt);
      finish_lists.push_back(f);
    }
    for (int s : fin) {
      slot_op[s] = -1;
      free_slots.push_back(s);
    }
    if (done_steps > max_steps)
      return fail(PPRS_ESTATE, "slot pool did not finish within %lld steps", max_steps);
  }
  // the last poll's results
  if (pack_over) return fail(PPRS_ESTATE, "pool upload exceeds its %zu bytes", pack_cap);
  if (pack_used > 0)
    HIPCHK(hipMemcpyAsync(dpack, hpack.data(), pack_used, hipMemcpyHostToDevice, c->stream));
  pack_used = 0;
  STCHK(launch_finish());
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->log) {
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    fprintf(stderr, "[pprs] pool of %d slots ran %d registrations in %lld steps, %.2f ms\n", S,
            n_ops, done_steps, ms);
    fflush(stderr);
  }
  return PPRS_OK;
}

// A scan element while a schedule's program runs on the host: the identity, or the result of
// registering frame k to frame i held in version `ver`.
struct ScanElem {
  bool ident;
  int i, k, ver;
};

// The schedule of a series as a program (pprs_scan_program): instructions, element count,
// operator applications and the widest level (in applications).
struct ScanProg {
  std::vector<int> code;
  int n_instr = 0, n_levels = 0, n_elems = 0, n_reg = 0, widest = 0;
};

pprs_status scan_program(const pprs_params* p, int M, ScanProg& sp) {
  sp = ScanProg{};
  if (M < 1) return PPRS_OK;
  if (pprs_scan_program(p->scan, M, p->scan_workers, nullptr, 0, &sp.n_instr, &sp.n_levels,
                        &sp.n_elems, &sp.n_reg) != PPRS_OK && sp.n_instr == 0)
    return fail(PPRS_EINVAL, "scan planning failed");
  sp.code.resize(5 * (size_t)std::max(sp.n_instr, 1));
  if (pprs_scan_program(p->scan, M, p->scan_workers, sp.code.data(), sp.n_instr, &sp.n_instr,
                        &sp.n_levels, &sp.n_elems, &sp.n_reg) != PPRS_OK)
    return fail(PPRS_EINVAL, "scan planning failed");
  std::vector<int> per_level(sp.n_levels + 1, 0);
  std::vector<char> ident(sp.n_elems, 1);
  for (int m = 0; m < M; ++m) ident[m] = 0;
  for (int t = 0; t < sp.n_instr; ++t) {
    const int* x = &sp.code[5 * (size_t)t];
    if (x[0] == PPRS_SCAN_OP_COMBINE) {
      if (!ident[x[1]] && !ident[x[2]]) per_level[x[4]]++;
      ident[x[3]] = ident[x[1]] && ident[x[2]];
    } else {
      ident[x[3]] = x[0] == PPRS_SCAN_OP_MOVE ? ident[x[1]] : 1;
    }
  }
  sp.widest = std::max(M, *std::max_element(per_level.begin(), per_level.end()));
  return PPRS_OK;
}

// Runs the program on the host: elements 0..M-1 start as the neighbour results (m, m+1) in
// versions ver0 + m, scratch elements as the identity. reg(left, right) is called for every
// operator application, in program order, and returns the version of its result. At the end
// element m must hold (0, m + 1); final (may be NULL) receives the elements.
template <class Reg>
pprs_status run_program(const ScanProg& sp, int M, int ver0, Reg reg,
                        std::vector<ScanElem>* final = nullptr) {
  std::vector<ScanElem> x(sp.n_elems, ScanElem{true, -1, -1, -1});
  for (int m = 0; m < M; ++m) x[m] = ScanElem{false, m, m + 1, ver0 + m};
  for (int t = 0; t < sp.n_instr; ++t) {
    const int* c = &sp.code[5 * (size_t)t];
    if (c[0] == PPRS_SCAN_OP_CLEAR) {
      x[c[3]] = ScanElem{true, -1, -1, -1};
    } else if (c[0] == PPRS_SCAN_OP_MOVE) {
      x[c[3]] = x[c[1]];
    } else if (x[c[1]].ident) {  // the identity costs nothing
      x[c[3]] = x[c[2]];
    } else if (x[c[2]].ident) {
      x[c[3]] = x[c[1]];
    } else {
      const ScanElem a = x[c[1]], b = x[c[2]];
      if (a.k != b.i)
        return fail(PPRS_EINDEX, "scan operands (%d,%d) and (%d,%d) do not share a frame", a.i,
                    a.k, b.i, b.k);
      x[c[3]] = ScanElem{false, a.i, b.k, reg(a, b)};
    }
  }
  for (int m = 0; m < M; ++m)
    if (x[m].ident || x[m].i != 0 || x[m].k != m + 1)
      return fail(PPRS_EINDEX, "element %d ends as (%d,%d)", m, x[m].i, x[m].k);
  if (final) *final = x;
  return PPRS_OK;
}

// Workspace of one cold pprs_prefix_register_series call of N frames of side H (level L,
// coarsest m0) on a pool of pool_slots slots: the bytes of every buffer it ensures, the slot
// count its pool takes and the slot layout (in hd). Mirrors run_series_set for one series.
struct SeriesWs {
  FrameBytes frames{};
  size_t elems = 0, pool_pack = 0, tmp = 0;
  SlotBytes slots{};
  int n_slots = 0;
  bool any = false;  // N > 1: the call allocates anything at all
  size_t total() const {
    if (!any) return 0;
    return frames.frames + frames.frame_off + frames.rsum + frames.fr_part + frames.fr_ms +
           frames.tcoef + elems + pool_pack + tmp + slots.state + slots.ubuf +
           slots.dbuf + slots.gbuf + slots.zbuf + slots.partial + slots.nodecount +
           slots.coef + slots.list_slots + slots.list_off + slots.lists + slots.desc +
           slots.opidx;
  }
};

pprs_status series_workspace(int N, int L, int m0, const pprs_params* p, int pool_slots,
                             BatchDesc& hd, SeriesWs& w) {
  w = SeriesWs{};
  int M = N - 1;
  if (M < 1) return PPRS_OK;
  w.any = true;
  size_t nodes = 0;
  for (int l = m0; l <= L; ++l) nodes += (size_t)N * level_n(l) * level_n(l);
  w.frames = frame_bytes(nodes, N, N);
  ScanProg sp;
  STCHK(scan_program(p, M, sp));
  int n_ops = sp.n_reg, widest = sp.widest;
  int nL = level_n(L);
  w.elems = sizeof(float) * (size_t)(M + n_ops) * 2 * nL * nL;
  int slots = std::min(widest, pool_slots);
  w.slots = slot_layout(hd, slots, L, m0, true);
  int S = std::max(1, std::min(slots, M + n_ops));
  w.n_slots = slots;
  w.pool_pack = pool_pack_bytes(S);
  w.tmp = sizeof(long long) * M;
  return PPRS_OK;
}

pprs_status series_args(int N, int H, int W, const pprs_params* params, int* L, int* m0) {
  *L = frame_level(H, W);
  if (*L < 0) return fail(PPRS_EINVAL, "frames must be square with side 2^L or 2^L+1, L in [2,10]");
  if (N < 1) return fail(PPRS_EINVAL, "N must be >= 1");
  STCHK(check_params(params, *L));
  *m0 = *L - params->levels + 1;
  return PPRS_OK;
}

pprs_status status_from_flags(int flags) {
  if (flags & PPRS_FLAG_NAN) return fail(PPRS_ENAN, "a registration produced a non-finite energy");
  if (flags & PPRS_FLAG_NONCONV) return PPRS_NOT_CONVERGED;
  return PPRS_OK;
}

pprs_status enter(pprs_ctx* c) {
  if (!c) return fail(PPRS_EINVAL, "ctx is NULL");
  HIPCHK(hipSetDevice(c->device));
  c->dlog_row0 = 0;
  return PPRS_OK;
}

}  // namespace

// ---- allocation-free pair registration ----------------------------------------------------
// pprs_register_pair_noalloc carves every buffer of one pair registration out of this array
// instead of allocating: frame staging and pyramids, the slot's fields, partial records and
// lists. Each device the library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for that device (the
// array's name is a host-side stand-in, not a device address).
#define PPRS_SCRATCH_BYTES (40u << 20)
static __device__ __align__(256) unsigned char scratch[PPRS_SCRATCH_BYTES];

namespace {

const int kMaxScratchDevices = 64;
void* g_scratch_dev[kMaxScratchDevices] = {nullptr};
std::mutex g_scratch_mu;

// Device address of `device`'s scratch array, looked up once per device with it current.
pprs_status scratch_for_device(int device, char** out) {
  if (device < 0 || device >= kMaxScratchDevices)
    return fail(PPRS_EINVAL, "device %d beyond the scratch table", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    HIPCHK(hipSetDevice(device));
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PPRS_EHIP, "no device address for the scratch array");
    g_scratch_dev[device] = p;
  }
  *out = (char*)g_scratch_dev[device];
  return PPRS_OK;
}

size_t align_up(size_t b) { return (b + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// Scratch a pair registration of H x W frames on levels m0..L carves (an upper bound: every
// buffer padded to the arena alignment), in the order pprs_register_pair ensures them.
size_t pair_scratch_bytes(int H, int W, int L, int m0) {
  int nL = level_n(L);
  size_t t = align_up(sizeof(float) * std::max((size_t)2 * H * W, (size_t)2 * nL * nL));
  size_t nodes = 0;
  for (int l = m0; l <= L; ++l) nodes += 2 * (size_t)level_n(l) * level_n(l);
  FrameBytes f = frame_bytes(nodes, 2, 2);
  t += align_up(f.frames) + align_up(f.frame_off) + align_up(f.rsum) + align_up(f.fr_part) +
       align_up(f.fr_ms) + align_up(f.tcoef);
  BatchDesc hd;
  memset(&hd, 0, sizeof hd);
  SlotBytes b = slot_layout(hd, 1, L, m0, true);
  for (size_t x : {b.state, b.ubuf, b.dbuf, b.gbuf, b.zbuf, b.partial, b.nodecount, b.coef,
                   b.list_slots, b.list_off, b.lists, b.desc, b.opidx})
    t += align_up(x);
  return t;
}

}  // namespace

// ---- C-ABI ---------------------------------------------------------------------------------

extern "C" {

void pprs_default_params(pprs_params* p) {
  if (!p) return;
  p->levels = 4;
  p->lambda = 10.0;
  p->beta = 1.0;
  p->armijo_sigma = 0.5;
  p->ladder_k = 1;
  p->step_cap = 1.0;
  p->tau_min_rel = 1e-4;
  p->eps = 3e-4;
  p->iter_max = 500;
  p->scan = PPRS_SCAN_BRENT_KUNG;
  p->scan_workers = 0;
  p->warm_start = 1;
  p->force_fallback = 0;
}

const char* pprs_last_error(void) { return g_err.c_str(); }

pprs_status pprs_create(pprs_ctx** out, int device, void* stream) {
  if (!out) return fail(PPRS_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  HIPCHK(hipGetDeviceCount(&count));
  if (device < 0 || device >= count)
    return fail(PPRS_EINVAL, "device %d out of range (%d devices)", device, count);
  HIPCHK(hipSetDevice(device));
  pprs_ctx* c = new pprs_ctx();
  memset(&c->hd, 0, sizeof(BatchDesc));
  c->device = device;
  const char* lg = getenv("PPRS_LOG");
  c->log = lg && lg[0] && lg[0] != '0';
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    // a blocking stream: ordered with the legacy default stream like the caller's work
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamDefault);
    if (e != hipSuccess) {
      delete c;
      return fail(PPRS_EHIP, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    c->own_stream = true;
  }
  hipError_t e = hipHostMalloc((void**)&c->active_host, sizeof(int), hipHostMallocDefault);
  if (e != hipSuccess) c->active_host = nullptr;
  char* sp = nullptr;
  pprs_status ss = scratch_for_device(device, &sp);  // once per device, this device current
  if (ss != PPRS_OK) {
    pprs_destroy(c);
    return ss;
  }
  *out = c;
  return PPRS_OK;
}

void pprs_destroy(pprs_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->active_host) (void)hipHostFree(c->active_host);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;  // every DevBuf frees its device memory
}

pprs_status pprs_workspace_query(int N, int H, int W, const pprs_params* params, size_t* bytes) {
  if (!bytes) return fail(PPRS_EINVAL, "bytes is NULL");
  int L, m0;
  STCHK(series_args(N, H, W, params, &L, &m0));
  BatchDesc hd;
  memset(&hd, 0, sizeof hd);
  SeriesWs w;
  STCHK(series_workspace(N, L, m0, params, kPoolSlotsDefault, hd, w));
  *bytes = w.total();
  return PPRS_OK;
}

pprs_status pprs_reserve_workspace(pprs_ctx* c, int N, int H, int W, const pprs_params* params) {
  STCHK(enter(c));
  int L, m0;
  STCHK(series_args(N, H, W, params, &L, &m0));
  BatchDesc hd;
  memset(&hd, 0, sizeof hd);
  SeriesWs w;
  STCHK(series_workspace(N, L, m0, params, c->pool_slots, hd, w));
  if (!w.any) return PPRS_OK;
  STCHK(ensure(c->frames, w.frames.frames));
  STCHK(ensure(c->frame_off, w.frames.frame_off));
  STCHK(ensure(c->rsum, w.frames.rsum));
  STCHK(ensure(c->fr_part, w.frames.fr_part));
  STCHK(ensure(c->fr_ms, w.frames.fr_ms));
  STCHK(ensure(c->tcoef, w.frames.tcoef));
  STCHK(ensure(c->elems, w.elems));
  STCHK(ensure(c->pool_pack, w.pool_pack));
  STCHK(ensure(c->tmp, w.tmp));
  STCHK(ensure_slots(c, w.n_slots, L, m0, params->beta));
  return PPRS_OK;
}

pprs_status pprs_workspace_bytes(pprs_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(PPRS_EINVAL, "NULL argument");
  size_t t = 0;
  for (const DevBuf* b : c->all_bufs()) t += b->p ? b->bytes : 0;
  *bytes = t;
  return PPRS_OK;
}

}  // extern "C"

namespace {

pprs_status register_pair_impl(pprs_ctx* c, const float* f_ref, const float* f_tmpl, int H,
                               int W, const float* u_init, float* u_out,
                               const pprs_params* params, pprs_pair_stats* stats) {
  int L = frame_level(H, W);
  if (L < 0) return fail(PPRS_EINVAL, "frames must be square with side 2^L or 2^L+1, L in [2,10]");
  if (!f_ref || !f_tmpl || !u_out) return fail(PPRS_EINVAL, "NULL frame or output pointer");
  STCHK(check_params(params, L));
  int m0 = L - params->levels + 1;
  int nL = level_n(L);
  size_t plane = (size_t)H * W;
  // stage both frames contiguously, then build the pyramids
  STCHK(ensure(c->elems, sizeof(float) * std::max(2 * plane, (size_t)2 * nL * nL)));
  float* stage = P<float>(c->elems);
  HIPCHK(hipMemcpyAsync(stage, f_ref, sizeof(float) * plane, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(stage + plane, f_tmpl, sizeof(float) * plane, hipMemcpyDeviceToDevice,
                        c->stream));
  STCHK(prepare_frames(c, stage, 2, H, L, m0, 1));
  STCHK(ensure_slots(c, 1, L, m0, params->beta));
  InitKind init = INIT_IDENTITY;
  if (u_init) {
    init = INIT_GIVEN;
    HIPCHK(pprs_k::to_nodes(u_init, H, (long long)plane, c->hd.ubuf + c->hd.u_off[L], nL,
                            (long long)nL * nL, 2, 1.0f / (float)(nL - 1), c->stream));
  }
  int ref = 0, tmpl = 1, out = 0;
  int flags = 0;
  STCHK(run_batch(c, 1, &ref, &tmpl, init, nullptr, nullptr, &out, stage, params, stats,
                  nullptr, nullptr, &flags));
  HIPCHK(pprs_k::from_nodes(stage, nL, (long long)nL * nL, u_out, H, (long long)plane, 2,
                            (float)(nL - 1), c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return status_from_flags(flags);
}

}  // namespace

extern "C" {

pprs_status pprs_register_pair(pprs_ctx* c, const float* f_ref, const float* f_tmpl, int H,
                               int W, const float* u_init, float* u_out,
                               const pprs_params* params, pprs_pair_stats* stats) {
  STCHK(enter(c));
  return register_pair_impl(c, f_ref, f_tmpl, H, W, u_init, u_out, params, stats);
}

pprs_status pprs_register_pair_noalloc(pprs_ctx* c, const float* f_ref, const float* f_tmpl,
                                       int H, int W, const float* u_init, float* u_out,
                                       const pprs_params* params, pprs_pair_stats* stats) {
  STCHK(enter(c));
  int L = frame_level(H, W);
  if (L < 0) return fail(PPRS_EINVAL, "frames must be square with side 2^L or 2^L+1, L in [2,10]");
  STCHK(check_params(params, L));
  size_t need = pair_scratch_bytes(H, W, L, L - params->levels + 1);
  if (need > PPRS_SCRATCH_BYTES)
    return fail(PPRS_EINVAL,
                "frames of %d x %d need %zu bytes of scratch; the allocation-free entry point "
                "has %u (frames up to 512 x 512)", H, W, need, PPRS_SCRATCH_BYTES);
  char* base = nullptr;
  STCHK(scratch_for_device(c->device, &base));
  // a context of the caller's stream and launch shape whose buffers all lie in the scratch
  pprs_ctx w;
  memset(&w.hd, 0, sizeof(BatchDesc));
  w.device = c->device;
  w.stream = c->stream;
  w.log = c->log;
  w.grid_energy = c->grid_energy;
  w.grid_grad = c->grid_grad;
  w.grid_smooth = c->grid_smooth;
  w.grid_prolong = c->grid_prolong;
  w.smooth_window = c->smooth_window;
  w.tile_grad = c->tile_grad;
  w.ladder_rungs = c->ladder_rungs;
  w.smooth_lines = c->smooth_lines;
  Arena arena{base, PPRS_SCRATCH_BYTES, 0, c->stream};
  g_arena = &arena;
  pprs_status s = register_pair_impl(&w, f_ref, f_tmpl, H, W, u_init, u_out, params, stats);
  g_arena = nullptr;
  return s;
}

pprs_status pprs_register_pairs(pprs_ctx* c, const float* frames, int N, int H, int W,
                                const int* ref, const int* tmpl, int P, float* u_out,
                                const pprs_params* params, pprs_pair_stats* stats) {
  STCHK(enter(c));
  int L = frame_level(H, W);
  if (L < 0) return fail(PPRS_EINVAL, "frames must be square with side 2^L or 2^L+1, L in [2,10]");
  if (!frames || !ref || !tmpl || !u_out || N < 1 || P < 0)
    return fail(PPRS_EINVAL, "bad arguments");
  STCHK(check_params(params, L));
  if (P == 0) return PPRS_OK;
  std::vector<char> is_ref(N, 0);
  for (int p = 0; p < P; ++p) {
    if (ref[p] < 0 || ref[p] >= N || tmpl[p] < 0 || tmpl[p] >= N)
      return fail(PPRS_EINVAL, "pair %d has a frame index out of range", p);
    is_ref[ref[p]] = 1;
  }
  int m0 = L - params->levels + 1;
  int nL = level_n(L);
  long long est = 2LL * nL * nL;
  size_t plane = (size_t)H * W;
  bool warm = c->cnn != nullptr && params->warm_start && m0 <= kWarmLevel && kWarmLevel <= L &&
              (c->warm_levels >> L & 1u);
  STCHK(prepare_frames(c, frames, N, H, L, m0, 0, &is_ref));
  int chunk = std::min(P, kPairChunk);
  STCHK(ensure(c->elems, sizeof(float) * est * chunk));
  STCHK(ensure_slots(c, chunk, L, m0, params->beta));
  float* elems = ::P<float>(c->elems);
  int flags = 0;
  for (int p0 = 0; p0 < P; p0 += chunk) {
    int np = std::min(chunk, P - p0);
    std::vector<int> out(np);
    for (int k = 0; k < np; ++k) out[k] = k;
    pprs_pair_stats* ps = stats ? stats + p0 : nullptr;
    c->dlog_row0 = p0;
    if (warm) {
      std::vector<int> lv, fl;
      STCHK(warm_init(c, np, ref + p0, tmpl + p0, m0, params->force_fallback != 0, lv, fl));
      STCHK(run_batch(c, np, ref + p0, tmpl + p0, INIT_PREPARED, nullptr, nullptr, out.data(),
                      elems, params, ps, nullptr, nullptr, &flags, m0, lv.data(), fl.data()));
    } else {
      STCHK(run_batch(c, np, ref + p0, tmpl + p0, INIT_IDENTITY, nullptr, nullptr, out.data(),
                      elems, params, ps, nullptr, nullptr, &flags));
    }
    HIPCHK(pprs_k::from_nodes(elems, nL, (long long)nL * nL, u_out + (size_t)p0 * 2 * plane, H,
                              (long long)plane, 2 * np, (float)(nL - 1), c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return status_from_flags(flags);
}

// Rigid variant of run_batch: n slots with parameters p0 (domain units, 3 per slot; NULL =
// identity) to completion; their parameters into p_out (host, 3 per slot).
pprs_status run_batch_rigid(pprs_ctx* c, int n, const int* ref, const int* tmpl,
                            const double* p0, double* p_out, const pprs_params* p,
                            pprs_pair_stats* stats, int* flags_or) {
  if (n <= 0) return PPRS_OK;
  auto t_start = std::chrono::steady_clock::now();
  BatchDesc& hd = c->hd;
  int L = hd.finest, m0 = hd.coarsest;
  hd.n_slots = n;
  hd.ladder_k = p->ladder_k;
  hd.rigid = 1;
  hd.lambda = 0.0;
  hd.sigma = p->armijo_sigma;
  hd.step_cap = p->step_cap;
  hd.tau_min_rel = p->tau_min_rel;
  hd.eps = p->eps;
  hd.iter_max = p->iter_max;
  STCHK(set_grad_tiles(c));
  // the rigid gradient pass works on the element tiles of the energy passes
  for (int l = m0; l <= L; ++l) hd.geom[l].tiles_grad = hd.geom[l].tiles_elem;
  BatchDesc* d = P<BatchDesc>(c->desc);
  hd.dlog = c->dlog ? c->dlog + (size_t)c->dlog_row0 * c->dlog_cap : nullptr;
  hd.dlog_cap = c->dlog_cap;
  HIPCHK(hipMemcpyAsync(d, &hd, sizeof(BatchDesc), hipMemcpyHostToDevice, c->stream));
  std::vector<SlotState> st(n);
  for (int s = 0; s < n; ++s) {
    memset(&st[s], 0, sizeof(SlotState));
    st[s].phase = PH_INIT;
    st[s].level = m0;
    st[s].ref = ref[s];
    st[s].tmpl = tmpl[s];
    st[s].finest = L;
    st[s].coarsest = m0;
    st[s].tau_prev = INFINITY;
    st[s].op = s;
    for (int k = 0; k < 3; ++k) st[s].rp[k] = p0 ? p0[3 * s + k] : 0.0;
  }
  HIPCHK(hipMemcpyAsync(hd.state, st.data(), sizeof(SlotState) * n, hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipMemsetAsync(hd.node_count, 0, sizeof(long long) * WK_COUNT * n, c->stream));
  int K = p->ladder_k, nc = ladder_rungs(c, K);
  long long max_steps = (long long)p->levels * ((long long)p->iter_max + 2) *
                            (ladder_pass_bound(p, nc) + 2) + 64;
  long long done_steps = 0;
  int group = 4;
  while (true) {
    for (int k = 0; k < group; ++k) STCHK(launch_step_rigid(c, d, nc));
    done_steps += group;
    int active = 0;
    HIPCHK(hipMemcpyAsync(&active, &d->active, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->timing) STCHK(tk_collect(c));
    if (active == 0) break;
    if (done_steps > max_steps) {
      hd.rigid = 0;
      return fail(PPRS_ESTATE, "rigid batch did not finish within %lld steps", max_steps);
    }
    group = std::min(group * 2, 32);
  }
  hd.rigid = 0;
  HIPCHK(hipMemcpyAsync(st.data(), hd.state, sizeof(SlotState) * n, hipMemcpyDeviceToHost,
                        c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  float batch_ms = (float)std::chrono::duration<double, std::milli>(
                       std::chrono::steady_clock::now() - t_start).count();
  for (int s = 0; s < n; ++s) {
    if (flags_or) *flags_or |= st[s].flags;
    for (int k = 0; k < 3; ++k) p_out[3 * s + k] = st[s].rp[k];
    if (stats) {
      pprs_pair_stats& o = stats[s];
      memset(&o, 0, sizeof o);
      for (int l = m0; l <= L; ++l) {
        o.iters[l - m0] = st[s].iters[l - m0];
        o.passes[l - m0] = st[s].passes[l - m0];
      }
      o.energy = st[s].E;
      o.ncc = st[s].ncc;
      o.flags = st[s].flags;
      o.ms = batch_ms;
    }
  }
  return PPRS_OK;
}

pprs_status pprs_register_pairs_rigid(pprs_ctx* c, const float* frames, int N, int H, int W,
                                      const int* ref, const int* tmpl, int P,
                                      const double* p_init, double* p_out,
                                      const pprs_params* params, pprs_pair_stats* stats) {
  STCHK(enter(c));
  int L = frame_level(H, W);
  if (L < 0) return fail(PPRS_EINVAL, "frames must be square with side 2^L or 2^L+1, L in [2,10]");
  if (!frames || !ref || !tmpl || !p_out || N < 1 || P < 0)
    return fail(PPRS_EINVAL, "bad arguments");
  STCHK(check_params(params, L));
  if (P == 0) return PPRS_OK;
  std::vector<char> is_ref(N, 0);
  for (int p = 0; p < P; ++p) {
    if (ref[p] < 0 || ref[p] >= N || tmpl[p] < 0 || tmpl[p] >= N)
      return fail(PPRS_EINVAL, "pair %d has a frame index out of range", p);
    is_ref[ref[p]] = 1;
  }
  int m0 = L - params->levels + 1;
  // API units: alpha in radians, t in pixels of the finest level (2^L per domain unit)
  const double px = (double)(level_n(L) - 1);
  STCHK(prepare_frames(c, frames, N, H, L, m0, 0, &is_ref));
  int chunk = std::min(P, kPairChunk);
  STCHK(ensure_slots(c, chunk, L, m0, params->beta, false));
  int flags = 0;
  std::vector<double> pin(3 * (size_t)chunk), pout(3 * (size_t)chunk);
  for (int p0 = 0; p0 < P; p0 += chunk) {
    int np = std::min(chunk, P - p0);
    for (int k = 0; k < np; ++k) {
      pin[3 * k] = p_init ? p_init[3 * (p0 + k)] : 0.0;
      pin[3 * k + 1] = p_init ? p_init[3 * (p0 + k) + 1] / px : 0.0;
      pin[3 * k + 2] = p_init ? p_init[3 * (p0 + k) + 2] / px : 0.0;
    }
    c->dlog_row0 = p0;
    STCHK(run_batch_rigid(c, np, ref + p0, tmpl + p0, pin.data(), pout.data(), params,
                          stats ? stats + p0 : nullptr, &flags));
    for (int k = 0; k < np; ++k) {
      p_out[3 * (p0 + k)] = pout[3 * k];
      p_out[3 * (p0 + k) + 1] = pout[3 * k + 1] * px;
      p_out[3 * (p0 + k) + 2] = pout[3 * k + 2] * px;
    }
  }
  return status_from_flags(flags);
}

pprs_status pprs_compose_deformations(pprs_ctx* c, const float* u_ij, const float* u_jk,
                                      float* u_ik, int H, int W) {
  STCHK(enter(c));
  int L = frame_level(H, W);
  if (L < 0) return fail(PPRS_EINVAL, "fields must be square with side 2^L or 2^L+1");
  if (!u_ij || !u_jk || !u_ik) return fail(PPRS_EINVAL, "NULL field pointer");
  int nL = level_n(L);
  long long est = 2LL * nL * nL;
  size_t plane = (size_t)H * W;
  STCHK(ensure(c->elems, sizeof(float) * 3 * est));
  STCHK(ensure(c->opidx, sizeof(int) * 3));
  float* e = P<float>(c->elems);
  float s = 1.0f / (float)(nL - 1);
  HIPCHK(pprs_k::to_nodes(u_ij, H, (long long)plane, e, nL, (long long)nL * nL, 2, s, c->stream));
  HIPCHK(pprs_k::to_nodes(u_jk, H, (long long)plane, e + est, nL, (long long)nL * nL, 2, s,
                          c->stream));
  int idx[3] = {0, 1, 0};
  int* didx = P<int>(c->opidx);
  HIPCHK(hipMemcpyAsync(didx, idx, sizeof idx, hipMemcpyHostToDevice, c->stream));
  HIPCHK(pprs_k::compose(e, est, didx, didx + 1, e + 2 * est, est, nL, 1, c->stream));
  HIPCHK(pprs_k::from_nodes(e + 2 * est, nL, (long long)nL * nL, u_ik, H, (long long)plane, 2,
                            (float)(nL - 1), c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return PPRS_OK;
}

// Rigid series (the series registration with the rigid operator): the N-1 neighbour
// registrations in one batch, then every level of the scan schedule as one batch, each B
// application started from the composition of its operands' maps,
// phi_jk o phi_ij: alpha = alpha_ij + alpha_jk, t = R(alpha_jk) t_ij + t_jk.
pprs_status pprs_prefix_register_series_rigid(pprs_ctx* c, const float* frames, int N, int H,
                                              int W, double* p_out, const pprs_params* params,
                                              pprs_series_stats* stats) {
  STCHK(enter(c));
  auto t0 = std::chrono::steady_clock::now();
  int L = frame_level(H, W);
  if (L < 0) return fail(PPRS_EINVAL, "frames must be square with side 2^L or 2^L+1, L in [2,10]");
  if (!frames || !p_out || N < 1) return fail(PPRS_EINVAL, "bad arguments");
  STCHK(check_params(params, L));
  for (int k = 0; k < 3; ++k) p_out[k] = 0.0;
  if (stats) memset(stats, 0, sizeof(*stats));
  int M = N - 1;
  if (M < 1) return PPRS_OK;
  int m0 = L - params->levels + 1;
  std::vector<char> is_ref(N, 1);
  STCHK(prepare_frames(c, frames, N, H, L, m0, 0, &is_ref));
  HIPCHK(hipStreamSynchronize(c->stream));
  auto t1 = std::chrono::steady_clock::now();
  int n_ops = 0, n_levels = 0;
  if (params->scan > PPRS_SCAN_GENERAL)
    return fail(PPRS_EINVAL, "the rigid series runs the in-place schedules (sequential, "
                "Brent-Kung, Kogge-Stone, Sklansky, general strategy)");
  pprs_scan_plan_p(params->scan, M, params->scan_workers, nullptr, 0, &n_ops, &n_levels);
  std::vector<int> plan(3 * (size_t)std::max(n_ops, 1));
  if (pprs_scan_plan_p(params->scan, M, params->scan_workers, plan.data(), n_ops, &n_ops,
                         &n_levels) != PPRS_OK)
    return fail(PPRS_EINVAL, "scan planning failed");
  int widest = M;
  for (int i = 0; i < n_ops;) {
    int j = i;
    while (j < n_ops && plan[3 * j + 2] == plan[3 * i + 2]) ++j;
    widest = std::max(widest, j - i);
    i = j;
  }
  STCHK(ensure_slots(c, widest, L, m0, params->beta, false));
  // elements x_m = (ei[m], ek[m], p[m]) in domain units
  std::vector<int> ei(M), ek(M), ref(widest), tmpl(widest);
  std::vector<double> pe(3 * (size_t)M), pin(3 * (size_t)widest), pres(3 * (size_t)widest);
  int flags = 0;
  for (int m = 0; m < M; ++m) {
    ei[m] = m;
    ek[m] = m + 1;
    ref[m] = m;
    tmpl[m] = m + 1;
  }
  STCHK(run_batch_rigid(c, M, ref.data(), tmpl.data(), nullptr, pe.data(), params, nullptr,
                        &flags));
  for (int i = 0; i < n_ops;) {
    int j = i;
    while (j < n_ops && plan[3 * j + 2] == plan[3 * i + 2]) ++j;
    int cnt = j - i;
    // operands as they stand before the level (within a level no op reads what another
    // op of the level writes)
    for (int q = 0; q < cnt; ++q) {
      int a = plan[3 * (i + q)], b = plan[3 * (i + q) + 1];
      if (ek[a] != ei[b])
        return fail(PPRS_EINDEX, "scan operands (%d,%d) and (%d,%d) do not share a frame", ei[a],
                    ek[a], ei[b], ek[b]);
      const double* u = &pe[3 * (size_t)a];  // phi_ij
      const double* v = &pe[3 * (size_t)b];  // phi_jk
      double cb = cos(v[0]), sb = sin(v[0]);
      pin[3 * q] = u[0] + v[0];
      pin[3 * q + 1] = cb * u[1] - sb * u[2] + v[1];
      pin[3 * q + 2] = sb * u[1] + cb * u[2] + v[2];
      ref[q] = ei[a];
      tmpl[q] = ek[b];
    }
    c->dlog_row0 = M + i;  // log rows: the M neighbour registrations, then B in schedule order
    STCHK(run_batch_rigid(c, cnt, ref.data(), tmpl.data(), pin.data(), pres.data(), params,
                          nullptr, &flags));
    for (int q = 0; q < cnt; ++q) {
      int a = plan[3 * (i + q)], b = plan[3 * (i + q) + 1];
      ei[b] = ei[a];
      for (int k = 0; k < 3; ++k) pe[3 * (size_t)b + k] = pres[3 * q + k];
    }
    i = j;
  }
  const double px = (double)(level_n(L) - 1);
  for (int m = 0; m < M; ++m) {
    if (ei[m] != 0 || ek[m] != m + 1)
      return fail(PPRS_EINDEX, "element %d ends as (%d,%d)", m, ei[m], ek[m]);
    p_out[3 * (m + 1)] = pe[3 * (size_t)m];
    p_out[3 * (m + 1) + 1] = pe[3 * (size_t)m + 1] * px;
    p_out[3 * (m + 1) + 2] = pe[3 * (size_t)m + 2] * px;
  }
  auto t2 = std::chrono::steady_clock::now();
  if (stats) {
    stats->n_ops_a = M;
    stats->n_ops_b = n_ops;
    stats->n_scan_levels = n_levels;
    stats->flags_or = flags;
    stats->ms_prepare = std::chrono::duration<double, std::milli>(t1 - t0).count();
    stats->ms_scan = std::chrono::duration<double, std::milli>(t2 - t1).count();
    stats->ms_total = std::chrono::duration<double, std::milli>(t2 - t0).count();
  }
  return status_from_flags(flags);
}

pprs_status pprs_series_average(pprs_ctx* c, const float* frames, const float* u, int N, int H,
                                int W, float* avg) {
  STCHK(enter(c));
  if (N < 1 || H < 2 || W < 2) return fail(PPRS_EINVAL, "need N >= 1 frames of at least 2x2");
  if (!frames || !u || !avg) return fail(PPRS_EINVAL, "NULL pointer");
  HIPCHK(pprs_k::series_average(frames, u, N, H, W, avg, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return PPRS_OK;
}

pprs_status pprs_series_average_refine(pprs_ctx* c, const float* frames, int N, int H, int W,
                                       float* u, int passes, const pprs_params* params,
                                       float* avg, pprs_pair_stats* stats) {
  STCHK(enter(c));
  int L = frame_level(H, W);
  if (L < 0) return fail(PPRS_EINVAL, "frames must be square with side 2^L or 2^L+1, L in [2,10]");
  if (!frames || !u || N < 1 || passes < 0) return fail(PPRS_EINVAL, "bad arguments");
  STCHK(check_params(params, L));
  int m0 = L - params->levels + 1;
  int nL = level_n(L);
  long long est = 2LL * nL * nL;
  size_t plane = (size_t)H * W;
  STCHK(ensure(c->avg_stage, sizeof(float) * plane));
  float* mean = P<float>(c->avg_stage);
  int n_pairs = N - 1;
  int chunk = std::max(1, std::min(n_pairs, kPairChunk));
  if (passes > 0 && n_pairs > 0) {
    STCHK(ensure(c->elems, sizeof(float) * est * chunk));
    STCHK(ensure_slots(c, chunk, L, m0, params->beta));
  }
  float* elems = P<float>(c->elems);
  // frames 0 .. N-1 are the templates, global frame N (the average) the one reference
  std::vector<char> no_ref(N, 0);
  std::vector<int> ref(chunk, N), tmpl(chunk), out(chunk);
  int flags = 0;
  for (int pass = 0; pass < passes && n_pairs > 0; ++pass) {
    HIPCHK(pprs_k::series_average(frames, u, N, H, W, mean, c->stream));
    std::vector<SeriesIn> ser{SeriesIn{frames, N, H, L, m0, 0, 0, &no_ref},
                              SeriesIn{mean, 1, H, L, m0, N, 1, nullptr}};
    STCHK(prepare_series(c, ser));
    for (int p0 = 0; p0 < n_pairs; p0 += chunk) {
      int np = std::min(chunk, n_pairs - p0);
      for (int k = 0; k < np; ++k) {
        tmpl[k] = 1 + p0 + k;
        out[k] = k;
      }
      // current deformations of frames 1+p0 .. on the finest level of the slots (domain units)
      float* u_src = u + (size_t)(1 + p0) * 2 * plane;
      HIPCHK(pprs_k::to_nodes(u_src, H, (long long)plane, elems, nL, (long long)nL * nL,
                              2 * np, 1.0f / (float)(nL - 1), c->stream));
      HIPCHK(hipMemcpy2DAsync(c->hd.ubuf + c->hd.u_off[L], sizeof(float) * c->hd.slot_u_stride,
                              elems, sizeof(float) * est, sizeof(float) * est, np,
                              hipMemcpyDeviceToDevice, c->stream));
      c->dlog_row0 = (long long)pass * n_pairs + p0;
      pprs_pair_stats* ps = stats ? stats + (size_t)pass * n_pairs + p0 : nullptr;
      STCHK(run_batch(c, np, ref.data(), tmpl.data(), INIT_GIVEN, nullptr, nullptr, out.data(),
                      elems, params, ps, nullptr, nullptr, &flags));
      HIPCHK(pprs_k::from_nodes(elems, nL, (long long)nL * nL, u_src, H, (long long)plane,
                                2 * np, (float)(nL - 1), c->stream));
    }
  }
  if (avg) HIPCHK(pprs_k::series_average(frames, u, N, H, W, avg, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return status_from_flags(flags);
}

// RAII for the series timing events.
struct EventSet {
  hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
  ~EventSet() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

// One series of a (possibly multi-series) registration run.
struct SeriesJob {
  const float* frames;  // device [N][H][H]
  int N, H, L, m0;
  float* u_out;         // device [N][2][H][H]
  pprs_series_stats* stats;
  pprs_pair_stats* op_stats;  // N-1 + B-op count entries, may be NULL
  double* latency_ms;   // time from the start of the run to the series' last result, or NULL
};

// Registers every series of `jobs` in one slot pool: the N-1 neighbour registrations and the
// scan's B applications of all series share the pool, each starting when its inputs exist.
pprs_status run_series_set(pprs_ctx* c, std::vector<SeriesJob>& jobs, const pprs_params* params) {
  EventSet ev;
  for (int k = 0; k < 4; ++k) HIPCHK(hipEventCreate(&ev.e[k]));
  HIPCHK(hipEventRecord(ev.e[0], c->stream));
  int Lmax = 0, m0min = PPRS_MAXL, f0 = 0, total_M = 0;
  std::vector<SeriesIn> sin;
  std::vector<int> first(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) {
    SeriesJob& x = jobs[j];
    size_t plane = (size_t)x.H * x.H;
    HIPCHK(pprs_k::fill(x.u_out, 2LL * (long long)plane, 0.f, c->stream));
    Lmax = std::max(Lmax, x.L);
    m0min = std::min(m0min, x.m0);
    first[j] = f0;
    if (x.N > 1) sin.push_back(SeriesIn{x.frames, x.N, x.H, x.L, x.m0, f0, x.N - 1, nullptr});
    f0 += x.N;
    total_M += std::max(0, x.N - 1);
  }
  if (!sin.empty()) STCHK(prepare_series(c, sin));
  HIPCHK(hipEventRecord(ev.e[1], c->stream));
  bool any_warm = c->cnn != nullptr && params->warm_start;
  // schedules: per series the scan program and the frame pairs of its B applications
  std::vector<ScanProg> progs(jobs.size());
  std::vector<std::vector<std::pair<int, int>>> bpairs(jobs.size());
  std::vector<int> n_ops_b(jobs.size(), 0), n_lv(jobs.size(), 0);
  int slots_needed = 1;
  for (size_t j = 0; j < jobs.size(); ++j) {
    int M = jobs[j].N - 1;
    if (M < 1) continue;
    STCHK(scan_program(params, M, progs[j]));
    n_ops_b[j] = progs[j].n_reg;
    n_lv[j] = progs[j].n_levels;
    slots_needed = std::max(slots_needed, progs[j].widest);
    auto& bp = bpairs[j];
    STCHK(run_program(progs[j], M, 0, [&](const ScanElem& a, const ScanElem& b) {
      bp.push_back({a.i, b.k});
      return 0;
    }));
  }
  // warm guesses, staged on level 7 for the neighbour pairs of every warm-capable series and,
  // where the series' finest level is above 7 (so that a level-7 judge can run), for the pairs
  // of its B applications too
  int n7 = level_n(kWarmLevel);
  long long per7 = 2LL * n7 * n7;
  PoolSpec spec;
  std::vector<int> stage_base(jobs.size(), -1);
  std::vector<char> judged(jobs.size(), 0);
  if (any_warm) {
    int nstage = 0;
    for (size_t j = 0; j < jobs.size(); ++j)
      if (jobs[j].m0 <= kWarmLevel && kWarmLevel <= jobs[j].L && jobs[j].N > 1 &&
          (c->warm_levels >> jobs[j].L & 1u)) {
        stage_base[j] = nstage;
        judged[j] = jobs[j].L > kWarmLevel;
        nstage += jobs[j].N - 1 + (judged[j] ? n_ops_b[j] : 0);
      }
    if (nstage > 0) {
      STCHK(ensure(c->warm_stage, sizeof(float) * per7 * nstage));
      spec.stage = P<float>(c->warm_stage);
      spec.stage_stride = per7;
      spec.stage_level = kWarmLevel;
    }
  }
  // the network runs before the registrations (its time is the "preprocess" figure)
  std::vector<std::vector<int>> bad(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) {
    if (stage_base[j] < 0) continue;
    int M = jobs[j].N - 1;
    std::vector<int> ref(M), tmpl(M);
    for (int m = 0; m < M; ++m) {
      ref[m] = m;
      tmpl[m] = m + 1;
    }
    if (judged[j])
      for (const auto& pr : bpairs[j]) {
        ref.push_back(pr.first);
        tmpl.push_back(pr.second);
      }
    STCHK(warm_predict(c, first[j], (int)ref.size(), ref.data(), tmpl.data(),
                       P<float>(c->warm_stage) + (size_t)stage_base[j] * per7, per7, bad[j],
                       params->force_fallback != 0));
  }
  HIPCHK(hipEventRecord(ev.e[2], c->stream));
  // op order is start priority: the cheapest series first (shortest job first keeps the
  // latency of short series low; the pool's throughput does not depend on the order)
  std::vector<int> order(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) order[j] = (int)j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    double ca = (double)jobs[a].N * level_n(jobs[a].L) * level_n(jobs[a].L);
    double cb = (double)jobs[b].N * level_n(jobs[b].L) * level_n(jobs[b].L);
    return ca < cb;
  });
  std::vector<PoolOp> ops;
  std::vector<long long> ver_off;
  std::vector<std::vector<int>> final_ver(jobs.size());
  std::vector<std::vector<int>> logical(jobs.size());  // pool op of each A, then B application
  std::vector<std::pair<int, int>> job_ops(jobs.size(), {0, 0});  // [first pool op, end)
  long long vtotal = 0;
  auto new_ver = [&](long long size) {
    ver_off.push_back(vtotal);
    vtotal += size;
    return (int)ver_off.size() - 1;
  };
  for (int j : order) {
    SeriesJob& x = jobs[j];
    int M = x.N - 1;
    job_ops[j] = {(int)ops.size(), (int)ops.size()};
    if (M < 1) continue;
    int nL = level_n(x.L);
    long long est = 2LL * nL * nL;
    int n_ops = n_ops_b[j];
    bool warm = stage_base[j] >= 0;
    bool skip = warm && c->warm_mode == PPRS_WARM_SKIP;
    int vb = (int)ver_off.size();
    for (int k = 0; k < M + n_ops; ++k) new_ver(est);
    int g0 = first[j];
    PoolOp base{0, 0, INIT_IDENTITY, -1, -1, -1, x.m0, 0, -1, x.L, x.m0};
    for (int m = 0; m < M; ++m) {
      PoolOp o = base;
      o.ref = g0 + m;
      o.tmpl = g0 + m + 1;
      o.out = vb + m;
      if (warm && bad[j][m]) {
        o.flags = PPRS_FLAG_FALLBACK;
      } else if (warm && !judged[j]) {
        o.init = INIT_PREPARED;
        o.stage = stage_base[j] + m;
        o.start = skip ? kWarmLevel : x.m0;
      } else if (warm) {
        // the judge: the warm registration up to level 7 (W) against the identity's NCC on
        // level 7 (I, evaluated only); the application resumes on level 8 from W's result, or
        // runs cold from the coarsest level when W ends with a lower NCC than the identity
        PoolOp w = o;
        w.init = INIT_PREPARED;
        w.stage = stage_base[j] + m;
        w.start = skip ? kWarmLevel : x.m0;
        w.stop = kWarmLevel;
        w.out = new_ver(per7);
        PoolOp id = o;
        id.start = kWarmLevel;
        id.stop = kWarmLevel;
        id.eval_only = 1;
        id.out = new_ver(per7);
        o.choose = CHOOSE_A;
        o.probe0 = (int)ops.size();
        o.probe1 = (int)ops.size() + 1;
        o.in0 = w.out;
        ops.push_back(w);
        ops.push_back(id);
      }
      logical[j].push_back((int)ops.size());
      ops.push_back(o);
    }
    // B applications in program order: (i, j, u) (.) (j, k, v) registers frame k to frame i,
    // starting from the composition of the two results
    int bi = 0;
    std::vector<ScanElem> fin;
    STCHK(run_program(progs[j], M, vb, [&](const ScanElem& l, const ScanElem& r) {
      int i = bi++;
      PoolOp o = base;
      o.ref = g0 + l.i;
      o.tmpl = g0 + r.k;
      o.init = INIT_COMPOSE;
      o.in0 = l.ver;
      o.in1 = r.ver;
      o.out = vb + M + i;
      o.start = skip ? kWarmLevel : x.m0;
      if (judged[j] && !bad[j][M + i]) {
        // the composition and the network's guess for the pair, both evaluated on level 7:
        // the start with the lower energy is taken
        PoolOp cp = o;
        cp.start = kWarmLevel;
        cp.stop = kWarmLevel;
        cp.eval_only = 1;
        cp.out = new_ver(per7);
        PoolOp nt = cp;
        nt.init = INIT_PREPARED;
        nt.in0 = nt.in1 = -1;
        nt.stage = stage_base[j] + M + i;
        nt.out = new_ver(per7);
        o.choose = CHOOSE_B;
        o.probe0 = (int)ops.size();
        o.probe1 = (int)ops.size() + 1;
        o.stage_alt = nt.stage;
        ops.push_back(cp);
        ops.push_back(nt);
      }
      logical[j].push_back((int)ops.size());
      ops.push_back(o);
      return o.out;
    }, &fin));
    for (int m = 0; m < M; ++m) final_ver[j].push_back(fin[m].ver);
    job_ops[j].second = (int)ops.size();
  }
  int flags = 0;
  long long node_steps = 0, node_passes = 0;
  std::vector<pprs_pair_stats> all_stats(ops.size());
  std::vector<double> fin_ms(ops.size(), 0.0);
  if (!ops.empty()) {
    int slots = std::min(slots_needed * (int)jobs.size(), c->pool_slots);
    STCHK(ensure(c->elems, sizeof(float) * std::max<long long>(vtotal, 1)));
    STCHK(ensure_slots(c, slots, Lmax, m0min, params->beta));
    float* vbuf = P<float>(c->elems);
    STCHK(run_pool(c, ops, slots, vbuf, ver_off, params, spec, all_stats.data(), &node_steps,
                   &node_passes, &flags, &fin_ms));
    for (size_t j = 0; j < jobs.size(); ++j) {
      SeriesJob& x = jobs[j];
      int M = x.N - 1;
      if (M < 1) continue;
      std::vector<long long> offs(M);
      for (int m = 0; m < M; ++m) offs[m] = ver_off[final_ver[j][m]];
      STCHK(ensure(c->tmp, sizeof(long long) * M));
      HIPCHK(hipMemcpyAsync(c->tmp.p, offs.data(), sizeof(long long) * M, hipMemcpyHostToDevice,
                            c->stream));
      size_t plane = (size_t)x.H * x.H;
      int nL = level_n(x.L);
      HIPCHK(pprs_k::from_nodes_idx(P<float>(c->elems), P<long long>(c->tmp), nL,
                                    x.u_out + 2 * plane, x.H, (long long)plane, M,
                                    (float)(nL - 1), c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
    }
  }
  HIPCHK(hipEventRecord(ev.e[3], c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
  (void)hipEventElapsedTime(&t01, ev.e[0], ev.e[1]);
  (void)hipEventElapsedTime(&t12, ev.e[1], ev.e[2]);
  (void)hipEventElapsedTime(&t23, ev.e[2], ev.e[3]);
  (void)hipEventElapsedTime(&t03, ev.e[0], ev.e[3]);
  for (size_t j = 0; j < jobs.size(); ++j) {
    SeriesJob& x = jobs[j];
    int a = job_ops[j].first, b = job_ops[j].second;
    pprs_series_stats S;
    memset(&S, 0, sizeof S);
    S.n_ops_a = std::max(0, x.N - 1);
    S.n_ops_b = n_ops_b[j];
    S.n_scan_levels = n_lv[j];
    double last = 0.0;
    for (int i = a; i < b; ++i) {  // every pool op of the series, probes included
      S.flags_or |= all_stats[i].flags;
      last = std::max(last, fin_ms[i]);
      for (int l = 0; l <= x.L - x.m0; ++l) {
        long long nn = (long long)level_n(x.m0 + l) * level_n(x.m0 + l);
        S.node_steps += nn * all_stats[i].iters[l];
        S.node_passes += nn * all_stats[i].passes[l];
      }
    }
    if (x.op_stats)
      for (size_t k = 0; k < logical[j].size(); ++k) {
        int f = logical[j][k];
        pprs_pair_stats o = all_stats[f];
        if (ops[f].init == INIT_RESUME) {  // levels up to 7 ran in the warm probe
          const pprs_pair_stats& w = all_stats[ops[f].probe0];
          for (int l = 0; l < ops[f].start - x.m0; ++l) {
            o.iters[l] = w.iters[l];
            o.passes[l] = w.passes[l];
          }
          o.flags |= w.flags;
          o.ms += w.ms;
        }
        x.op_stats[k] = o;
      }
    S.ms_total = t03;
    S.ms_prepare = t01;
    S.ms_preprocess = t12;
    S.ms_scan = t23;
    if (x.stats) *x.stats = S;
    if (x.latency_ms) *x.latency_ms = t01 + t12 + last;
  }
  return status_from_flags(flags);
}

pprs_status pprs_prefix_register_series(pprs_ctx* c, const float* frames, int N, int H, int W,
                                        float* u_out, const pprs_params* params,
                                        pprs_series_stats* stats, pprs_pair_stats* op_stats) {
  STCHK(enter(c));
  int L = frame_level(H, W);
  if (L < 0) return fail(PPRS_EINVAL, "frames must be square with side 2^L or 2^L+1, L in [2,10]");
  if (N < 1) return fail(PPRS_EINVAL, "N must be >= 1");
  if (!frames || !u_out) return fail(PPRS_EINVAL, "NULL frames or output pointer");
  STCHK(check_params(params, L));
  std::vector<SeriesJob> jobs{SeriesJob{frames, N, H, L, L - params->levels + 1, u_out, stats,
                                        op_stats, nullptr}};
  return run_series_set(c, jobs, params);
}

pprs_status pprs_register_series_batch(pprs_ctx* c, int S, const float* const* frames,
                                       const int* N, const int* side, const int* levels,
                                       float* const* u_out, const pprs_params* params,
                                       pprs_series_stats* stats, double* latency_ms) {
  STCHK(enter(c));
  if (S < 1 || !frames || !N || !side || !u_out || !params)
    return fail(PPRS_EINVAL, "bad arguments");
  std::vector<SeriesJob> jobs;
  for (int j = 0; j < S; ++j) {
    int L = frame_level(side[j], side[j]);
    if (L < 0) return fail(PPRS_EINVAL, "series %d: side must be 2^L or 2^L+1, L in [2,10]", j);
    if (N[j] < 1 || !frames[j] || !u_out[j]) return fail(PPRS_EINVAL, "series %d: bad arguments", j);
    pprs_params pj = *params;
    if (levels) pj.levels = levels[j];
    STCHK(check_params(&pj, L));
    jobs.push_back(SeriesJob{frames[j], N[j], side[j], L, L - pj.levels + 1, u_out[j],
                             stats ? stats + j : nullptr, nullptr,
                             latency_ms ? latency_ms + j : nullptr});
  }
  return run_series_set(c, jobs, params);
}

pprs_status pprs_prefix_register_series_batch(pprs_ctx* c, int S, const float* const* frames,
                                              const int* N, const int* H, const int* W,
                                              float* const* u_out, const pprs_params* params,
                                              pprs_series_stats* stats) {
  if (S < 1 || !H || !W) return fail(PPRS_EINVAL, "bad arguments");
  for (int j = 0; j < S; ++j)
    if (H[j] != W[j]) return fail(PPRS_EINVAL, "series %d: frames must be square", j);
  return pprs_register_series_batch(c, S, frames, N, H, nullptr, u_out, params, stats, nullptr);
}

pprs_status pprs_set_decision_log(pprs_ctx* c, unsigned char* log, int cap) {
  if (!c) return fail(PPRS_EINVAL, "ctx is NULL");
  if (log && cap < 1) return fail(PPRS_EINVAL, "cap must be >= 1");
  c->dlog = log;
  c->dlog_cap = log ? cap : 0;
  return PPRS_OK;
}

pprs_status pprs_set_metric_solve(pprs_ctx* c, int mode) {
  if (!c) return fail(PPRS_EINVAL, "ctx is NULL");
  if (mode != PPRS_METRIC_EXACT && mode != PPRS_METRIC_WINDOW)
    return fail(PPRS_EINVAL, "unknown metric-solve mode %d", mode);
  bool w = mode == PPRS_METRIC_WINDOW;
  if (w != c->smooth_window) {
    c->smooth_window = w;
    c->coef_beta = -1.0;  // recompute the coefficients and the halo on the next call
  }
  return PPRS_OK;
}

pprs_status pprs_get_tuning(pprs_ctx* c, pprs_tuning* t) {
  if (!c || !t) return fail(PPRS_EINVAL, "NULL argument");
  t->pool_slots = c->pool_slots;
  t->pool_group = c->pool_group;
  t->grid_energy = c->grid_energy;
  t->grid_grad = c->grid_grad;
  t->grid_smooth = c->grid_smooth;
  t->grid_prolong = c->grid_prolong;
  t->tile_grad = c->tile_grad;
  t->smooth_lines = c->smooth_lines;
  t->ladder_rungs = c->ladder_rungs;
  return PPRS_OK;
}

pprs_status pprs_set_tuning(pprs_ctx* c, const pprs_tuning* t) {
  if (!c || !t) return fail(PPRS_EINVAL, "NULL argument");
  const int v[8] = {t->pool_slots, t->pool_group, t->grid_energy, t->grid_grad, t->grid_smooth,
                    t->grid_prolong, t->tile_grad, t->smooth_lines};
  const int hi[8] = {65536, 1024, 65536, 65536, 65536, 65536, 4, 32};
  for (int k = 0; k < 8; ++k)
    if (v[k] < 0 || v[k] > hi[k]) return fail(PPRS_EINVAL, "tuning value %d out of range", k);
  c->pool_slots = t->pool_slots ? t->pool_slots : 512;
  c->pool_group = t->pool_group ? t->pool_group : 16;
  c->grid_energy = t->grid_energy ? t->grid_energy : 8192;
  c->grid_grad = t->grid_grad ? t->grid_grad : 8192;
  c->grid_smooth = t->grid_smooth ? t->grid_smooth : 8192;
  c->grid_prolong = t->grid_prolong ? t->grid_prolong : 2048;
  c->tile_grad = t->tile_grad;
  if (t->smooth_lines != 0 && t->smooth_lines != 8 && t->smooth_lines != 16 &&
      t->smooth_lines != 32)
    return fail(PPRS_EINVAL, "smooth_lines must be 8, 16 or 32");
  c->smooth_lines = t->smooth_lines ? t->smooth_lines : 16;
  if (t->ladder_rungs != 0 && !pprs_k::ladder_rungs_ok(t->ladder_rungs))
    return fail(PPRS_EINVAL, "ladder_rungs must be 0, 1, 2, 3, 5 or 7");
  c->ladder_rungs = t->ladder_rungs;
  return PPRS_OK;
}

pprs_status pprs_set_pool(pprs_ctx* c, int slots, int group_steps) {
  STCHK(enter(c));
  if (slots < 0 || group_steps < 0 || slots > 65536 || group_steps > 1024)
    return fail(PPRS_EINVAL, "slots must be in [0, 65536] and group_steps in [0, 1024]");
  c->pool_slots = slots ? slots : 512;
  c->pool_group = group_steps ? group_steps : 16;
  return PPRS_OK;
}

pprs_status pprs_set_warm_sides(pprs_ctx* c, unsigned level_mask) {
  STCHK(enter(c));
  c->warm_levels = level_mask;
  return PPRS_OK;
}

pprs_status pprs_set_warm_start(pprs_ctx* c, pprs_cnn* cnn, double max_cells, int mode) {
  STCHK(enter(c));
  if (mode != PPRS_WARM_REFINE && mode != PPRS_WARM_SKIP)
    return fail(PPRS_EINVAL, "unknown warm-start mode %d", mode);
  if (cnn && pprs_cnn_api::cnn_device(cnn) != c->device)
    return fail(PPRS_EINVAL, "network and context are on different devices");
  if (!(max_cells > 0.0)) return fail(PPRS_EINVAL, "max_cells must be > 0");
  c->cnn = cnn;
  c->warm_max_cells = max_cells;
  c->warm_mode = mode;
  return PPRS_OK;
}

pprs_status pprs_pair_inputs(pprs_ctx* c, const float* frames, int N, int H, int W,
                             const int* ref, const int* tmpl, int P, float* out) {
  STCHK(enter(c));
  int L = frame_level(H, W);
  if (L < kWarmLevel) return fail(PPRS_EINVAL, "frames must have a side of at least 128");
  if (!frames || !ref || !tmpl || !out || N < 1 || P < 1) return fail(PPRS_EINVAL, "bad arguments");
  for (int p = 0; p < P; ++p)
    if (ref[p] < 0 || ref[p] >= N || tmpl[p] < 0 || tmpl[p] >= N)
      return fail(PPRS_EINVAL, "pair %d has a frame index out of range", p);
  STCHK(prepare_frames(c, frames, N, H, L, kWarmLevel, 0));
  STCHK(ensure(c->badflags, sizeof(int) * 2 * (size_t)P));
  int* dref = ::P<int>(c->badflags);
  HIPCHK(hipMemcpyAsync(dref, ref, sizeof(int) * P, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(dref + P, tmpl, sizeof(int) * P, hipMemcpyHostToDevice, c->stream));
  int S = 1 << kWarmLevel;
  HIPCHK(pprs_cnn_api::pack_pairs(frame_level_ptr(c, 0, kWarmLevel), S + 1, dref, dref + P, P, out,
                                  c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return PPRS_OK;
}

pprs_status pprs_level7_targets(pprs_ctx* c, const float* u, int P, int H, int W, float* out) {
  STCHK(enter(c));
  int L = frame_level(H, W);
  if (L < kWarmLevel) return fail(PPRS_EINVAL, "fields must have a side of at least 128");
  if (!u || !out || P < 1) return fail(PPRS_EINVAL, "bad arguments");
  int nL = level_n(L);
  const int chunk = 256;
  // per chunk: level L planes, then the restrictions down to level 7 (ping-pong)
  size_t a = (size_t)2 * chunk * nL * nL, b = (size_t)2 * chunk * level_n(L - 1) * level_n(L - 1);
  STCHK(ensure(c->tmp, sizeof(float) * (a + b)));
  float* bufA = ::P<float>(c->tmp);
  float* bufB = bufA + a;
  size_t plane = (size_t)H * W;
  int S = 1 << kWarmLevel;
  for (int p0 = 0; p0 < P; p0 += chunk) {
    int np = std::min(chunk, P - p0);
    HIPCHK(pprs_k::to_nodes(u + (size_t)p0 * 2 * plane, H, (long long)plane, bufA, nL,
                            (long long)nL * nL, 2 * np, 1.0f / (float)(nL - 1), c->stream));
    float* cur = bufA;
    float* nxt = bufB;
    for (int l = L; l > kWarmLevel; --l) {
      int nf = level_n(l), nc = level_n(l - 1);
      HIPCHK(pprs_k::restrict_planes(cur, (long long)nf * nf, 0, nxt, (long long)nc * nc, 0, 1,
                                     nf, 2 * np, c->stream));
      std::swap(cur, nxt);
    }
    HIPCHK(pprs_cnn_api::planes_to_nhwc(cur, S + 1, 2LL * (S + 1) * (S + 1), np, (float)S,
                                        out + (size_t)p0 * S * S * 2, c->stream));
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  return PPRS_OK;
}

pprs_status pprs_set_kernel_timing(pprs_ctx* c, int enable) {
  STCHK(enter(c));
  c->timing = enable != 0;
  return PPRS_OK;
}

pprs_status pprs_get_kernel_timing(pprs_ctx* c, double* ms, long long* launches, double* bytes,
                                   int cap, int* n_kinds, int reset) {
  if (!c) return fail(PPRS_EINVAL, "ctx is NULL");
  if (n_kinds) *n_kinds = TK_COUNT;
  // node counts per work kind -> bytes per timing kind
  const int wk_of_tk[TK_COUNT] = {-1, WK_PROLONG, WK_EVAL, WK_GRAD, WK_SMY, WK_SMX, WK_LADDER,
                                  -1, WK_SMX};
  for (int k = 0; k < TK_COUNT && k < cap; ++k) {
    if (ms) ms[k] = c->t_ms[k];
    if (launches) launches[k] = c->t_launch[k];
    // the metric solve counts its nodes under WK_SMX in both forms: bytes go to the form
    // that ran
    if (bytes)
      bytes[k] = wk_of_tk[k] < 0 || c->t_launch[k] == 0
                     ? 0.0 : kBytesPerNode[k] * c->nodes_acc[wk_of_tk[k]];
  }
  // the field path runs the start energies inside the line-search launches and the
  // prolongations inside the gradient launches: their bytes belong to those kinds
  if (bytes && TK_LADDER < cap && c->t_launch[TK_EVAL] == 0 && c->t_launch[TK_LADDER] > 0)
    bytes[TK_LADDER] += kBytesPerNode[TK_EVAL] * c->nodes_acc[WK_EVAL];
  if (bytes && TK_GRAD < cap && c->t_launch[TK_PROLONG] == 0 && c->t_launch[TK_GRAD] > 0)
    bytes[TK_GRAD] += kBytesPerNode[TK_PROLONG] * c->nodes_acc[WK_PROLONG];
  if (reset) {
    for (int k = 0; k < TK_COUNT; ++k) {
      c->t_ms[k] = 0;
      c->t_launch[k] = 0;
    }
    for (int k = 0; k < WK_COUNT; ++k) c->nodes_acc[k] = 0;
  }
  return PPRS_OK;
}

const char* pprs_kernel_name(int kind) {
  if (kind < 0 || kind >= TK_COUNT) return "unknown";
  return kTkName[kind];
}

}  // extern "C"
