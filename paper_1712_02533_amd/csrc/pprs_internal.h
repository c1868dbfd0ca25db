// Internal data structures shared by the HIP kernels and the host runtime of libpprs.
//
// Discrete method (one reading of the paper's "Image registration for electron microscopy"
// section, identical to the one the FP64 oracle follows):
//   level l: n = 2^l + 1 nodes per axis, h = 1/(n-1); node (a, b) at (b h, a h).
//   u: nodal displacement in domain units, two planes (x, y).
//   NCC integrals: 2x2 Gauss rule per element, template composed at the quadrature points.
//   E(u) = -NCC + (lambda/2) sum_c u_c^T K u_c,  K = Q1 stiffness.
//   gradient flow: d = A^{-1} G, A = S1 (x) S1, S1 = M1 + (beta h)^2 K1; Armijo ladder.
#pragma once
#include <stdint.h>

#define PPRS_MAXL 16

// Slot phases. A slot is one application of A (or of the registration part of B).
enum {
  PH_DONE = 0,
  PH_INIT = 1,     // energy of the starting u at the current level is needed
  PH_GRAD = 2,     // gradient + metric solve for the current accepted u
  PH_LADDER = 3,   // one line-search pass
  PH_PROLONG = 4,  // level finished; prolongate to level + 1 (which then needs its energy)
};

// Work kinds of the per-step kernels (one item list each).
enum { WK_PROLONG = 0, WK_EVAL = 1, WK_GRAD = 2, WK_SMY = 3, WK_SMX = 4, WK_LADDER = 5,
       WK_COUNT = 6 };

// Tile geometry (compile-time).
#define ET_X 64   // energy kernel: elements per tile along x
#define ET_Y 16   //                elements per tile along y
#define PT_X 64   // prolongation: fine nodes per tile along x
#define PT_Y 8
// smoother: lines per workgroup, chosen per level so one strip stays under 40 KB of LDS
#define SM_LDS_MAX_FLOATS 33825  // column-solve strip in LDS: n (lines + 1) floats, <= 135 KB
#define SW_T 64          // windowed metric solve: output nodes per tile along each axis
#define SW_THREADS 128
#define SM_THREADS 256
#define BLOCK 256
#define MAX_CAND 7      // 2K+1 with K <= 3

// Per-slot state, in device memory. All floating-point scalars are FP64.
struct SlotState {
  int phase;
  int level;     // current absolute level
  int ub;        // which of the two u buffers of the current level holds u
  int iter;      // accepted steps on the current level
  int flags;     // PPRS_FLAG_*
  int ref;       // reference frame index
  int tmpl;      // template frame index
  int finest;    // L
  int coarsest;  // m0
  int rung;      // index, within its group of 2K+1 steps, of the pending pass's first step
  int op;        // row of the registration in the call's decision log (BatchDesc::dlog)
  int eval_only; // probe: evaluate the start energy on the start level, then stop
  double E;      // energy at the accepted u (= u[ub] - tau_pend d)
  double ncc;
  double mean;   // quadrature mean of the warped template at the accepted u
  double sigma;  // quadrature std of the warped template at the accepted u
  double tau_prev;
  double top;
  double tau_max;
  double tau_pend;  // accepted step not yet applied to u[ub]
  double gtd;
  double dmax;
  double rp[3];  // rigid variant: alpha, t0, t1 (domain units) of phi(x) = R(alpha) x + t
  double rd[3];  // rigid variant: search direction in the parameters
  int iters[PPRS_MAXL];
  int passes[PPRS_MAXL];
};

// Geometry of one level (host-filled, device-read).
struct LevelGeom {
  int n;
  int tiles_grad;   // gradient tiles of the chosen tile shape (tile_grad variant)
  int tiles_elem;   // ceil((n-1)/ET_X) * ceil((n-1)/ET_Y)
  int tiles_prol;   // ceil(n/PT_X) * ceil(n/PT_Y) (fine-level tiles when this is the target)
  int sm_lines;     // lines per smoother workgroup
  int sm_items;     // ceil(n / sm_lines) per component
  int coef_off;     // offset of this level's smoother coefficients
  int sw_tiles;     // windowed metric solve: tiles per axis (max(1, (n-1) / SW_T))
};

// Per-kind item list built by the planning kernel each step.
struct WorkList {
  int n_slots;   // slots in the list
  int total;     // total items
};

// Everything the per-step kernels need; lives in device memory, pointers fixed per context.
// Row pitch (floats) of a level's gradient and metric-solve buffers: rows start on 128-byte
// lines, so the column-strip solve reads and writes whole lines instead of straddling two.
#define WPAD 32
__host__ __device__ inline int row_pitch(int n) { return (n + WPAD - 1) / WPAD * WPAD; }
// Entries per coefficient array of a level's line solves: n rounded up to whole 64-lane chunks.
__host__ __device__ inline int coef_pitch(int n) { return (n + 63) / 64 * 64; }

struct BatchDesc {
  int n_slots;
  int finest;
  int coarsest;
  int ladder_k;
  double lambda;
  double sigma;
  double step_cap;
  double tau_min_rel;
  double eps;
  int iter_max;
  int smooth_halo;         // windowed metric solve halo in nodes; 0: exact two-pass line solves
  int rigid;               // 1: the slots run the rigid variant (parameters rp, no fields)
  LevelGeom geom[PPRS_MAXL];
  // frames: normalised pyramids; frame f at level l starts at pyr + frame_off[f][l]
  float* pyr;
  const long long* frame_off;  // [frame][PPRS_MAXL] offsets in floats (-1: level not built)
  double* rsum;            // [frame][PPRS_MAXL]: quadrature integral of the normalised frame
  // slots
  SlotState* state;        // [n_slots]
  float* ubuf;             // slot s: ubuf + s * slot_u_stride; level l at u_off[l]
  long long slot_u_stride;
  long long u_off[PPRS_MAXL];  // offset of level l: [2 buffers][2 comps][n_l^2]
  float* dbuf;             // [slot][2][nL^2] search direction
  float* gbuf;             // [slot][2][nL][row_pitch(nL)] gradient (rows padded, see row_pitch)
  float* zbuf;             // [slot][2][nL][row_pitch(nL)] metric solve intermediate
  long long slot_f_stride; // 2 * nL^2
  long long slot_p_stride; // 2 * nL * row_pitch(nL)
  double* partial;         // [slot][kind][max_items][PW]
  long long part_slot_stride;
  long long part_kind_stride;
  long long* node_count;   // [slot][WK_COUNT] grid nodes processed per kind (statistics)
  // smoother coefficients: inv_den[i], cprime[i] per level (float)
  float* coef;
  // per-step item lists
  int* list_slots;         // [WK_COUNT][max_slots]
  int* list_off;           // [WK_COUNT][max_slots + 1]
  WorkList* lists;         // [WK_COUNT]
  int max_slots;
  // decision log (optional, caller's device buffer): row op, entry k = ladder position J of the
  // op's k-th accepted step (levels in order), the step being top 2^-J of its iteration
  unsigned char* dlog;
  int dlog_cap;
  float* tcoef;            // per pyramid node (same offsets x 4): v, v(+x) - v, v(+y) - v,
                           // v(+x+y) - v(+y) - v(+x) + v (0 past the last row / column)
  int active;              // written by the plan kernel
  int* active_host;        // mapped host word (may be null)
};

#define PW 24   // doubles per partial record (3 * MAX_CAND + 3)
