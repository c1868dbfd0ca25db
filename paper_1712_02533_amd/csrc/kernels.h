// Launch wrappers of the HIP kernels (kernels.hip). All take the context stream.
#pragma once
#include <hip/hip_runtime.h>
#include "pprs_internal.h"

namespace pprs_k {
hipError_t plan(BatchDesc* d, hipStream_t st);
// nc: step sizes per line-search pass (1, 2, 3, 5 or 7; ladder_rungs_ok)
bool ladder_rungs_ok(int nc);
// start energies (eval list) and line-search passes (ladder list) of a step in one launch,
// and their finalisers
hipError_t energy_step(BatchDesc* d, int nc, int grid, hipStream_t st);
hipError_t energy_step_fin(BatchDesc* d, int nc, int grid, hipStream_t st);
hipError_t smooth_fin(BatchDesc* d, int grid, hipStream_t st);
// gradient tile variants: 0 = 32x16, 1 = 64x8, 2 = 128x4, 3 = 64x16 nodes
void grad_tile(int variant, int* tx, int* ty);
hipError_t grad(BatchDesc* d, int variant, int grid, hipStream_t st);
hipError_t smooth(BatchDesc* d, int dir, bool big, int grid, size_t lds_bytes, hipStream_t st);
hipError_t set_smooth_lds(size_t bytes);
// windowed metric solve (both axes in one launch); halo 16 or 24
hipError_t smooth_win(BatchDesc* d, int halo, int grid, hipStream_t st);
hipError_t restrict_planes(const float* src, long long s_outer, long long s_inner, float* dst,
                           long long d_outer, long long d_inner, int inner, int nf, int planes,
                           hipStream_t st);
hipError_t to_nodes(const float* src, int H, long long s_plane, float* dst, int n,
                    long long d_plane, int planes, float scale, hipStream_t st);
hipError_t from_nodes(const float* src, int n, long long s_plane, float* dst, int H,
                      long long d_plane, int planes, float scale, hipStream_t st);
hipError_t fill(float* p, long long count, float v, hipStream_t st);
// bilinear coefficients of N frames of n x n nodes (frame stride n^2) into 4 floats per node
hipError_t tcoef(const float* f, int n, int N, float* coef, hipStream_t st);
hipError_t fill_strided(float* p, long long outer, long long per, int n_outer, float v,
                        hipStream_t st);
hipError_t elem_sums(const float* src, long long plane_stride, int n, int bands, int planes,
                     double* partial, hipStream_t st);
hipError_t elem_final(const double* partial, int bands, int planes, int mode, double* ms,
                      double* rsum, int rs_stride, int rs_off, hipStream_t st);
hipError_t normalize(float* f, long long plane_stride, long long per_plane, int planes,
                     const double* ms, hipStream_t st);
hipError_t compose(const float* elems, long long estride, const int* left_idx,
                   const int* right_idx, float* out_base, long long ostride, int n, int ops,
                   hipStream_t st);
hipError_t finish(BatchDesc* d, const int* out_idx, float* elems, long long estride,
                  long long work, hipStream_t st);
// slot pool (index-list addressing)
hipError_t pool_assign(BatchDesc* d, const SlotState* staged, const int* slots, int ops,
                       hipStream_t st);
hipError_t pool_zero(BatchDesc* d, int l, int n_l, const int* slots, int ops, hipStream_t st);
hipError_t pool_compose(BatchDesc* d, int L, const float* vbuf, const long long* off0,
                        const long long* off1, const int* slots, int ops, hipStream_t st);
hipError_t pool_restrict(BatchDesc* d, int l, int n_c, const int* slots, int ops,
                         hipStream_t st);
hipError_t pool_copy(BatchDesc* d, int l, int n_l, const float* src, long long sstride,
                     const int* src_idx, const int* slots, int ops, hipStream_t st);
hipError_t pool_copy_off(BatchDesc* d, int l, int n_l, const float* vbuf, const long long* offs,
                         const int* slots, int ops, hipStream_t st);
hipError_t pool_finish(BatchDesc* d, int L, const int* slots, const long long* outs, int ops,
                       float* vbuf, hipStream_t st);
hipError_t from_nodes_idx(const float* vbuf, const long long* offs, int n, float* dst, int H,
                          long long d_plane, int elems, float scale, hipStream_t st);
// rigid variant: energy passes (mode 0 start, 1 line search with nc steps), gradient, its
// per-slot finaliser (the energy finalisers are energy_fin's)
// start energies (eval list) and line-search passes (ladder list) of the rigid slots, one launch
hipError_t rigid_energy_step(BatchDesc* d, int nc, int grid, hipStream_t st);
hipError_t rigid_grad(BatchDesc* d, int grid, hipStream_t st);
hipError_t rigid_grad_fin(BatchDesc* d, int grid, hipStream_t st);
// avg[H][W] = mean over i of frames[i] sampled at x + u[i](x) (pixels, clamped, bilinear)
hipError_t series_average(const float* frames, const float* u, int N, int H, int W, float* out,
                          hipStream_t st);
}  // namespace pprs_k
