/*
 * FP64 CPU oracle of the multilevel gradient-flow registration operator and of the series
 * prefix scan (Copik 2017, "Image registration" and "Prefix sum" chapters).
 *
 * TEST INFRASTRUCTURE ONLY. It is plain, slow and written to be checked against the paper by
 * eye: every step follows the formula it implements, with no blocking, fusion or reordering.
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may load it;
 * the product path never calls it and shares no code with it.
 *
 * Grids (Multilevel section): level l has n = 2^l + 1 nodes per axis, spacing h = 1/(n-1),
 * node (a, b) (row a, column b) at the point (x, y) = (b h, a h) of the unit square. Nodal
 * arrays are row-major [a][b]. A displacement u = phi - id is stored as two planes (x then y)
 * in domain units.
 *
 * Readings taken where the paper is silent or garbled (each one is listed in the design notes):
 *  - restriction at the border: the full-weighting stencil truncated to in-range nodes and
 *    renormalised;
 *  - prolongation: the standard vertex-centred bilinear rule (the figure caption says bilinear;
 *    the printed case table is garbled);
 *  - sampling outside the domain: clamp (replicate), derivative of the clamped function;
 *  - mass matrix: the consistent Q1 matrix M = M1 (x) M1; stiffness K = K1 (x) M1 + M1 (x) K1;
 *  - metric of the gradient flow: A = S1 (x) S1 with S1 = M1 + (beta h)^2 K1;
 *  - Armijo rule: Phi(tau) <= Phi(0) + sigma tau Phi'(0) with Phi'(0) = -G.d, evaluated on a
 *    ladder of 2K+1 step sizes top * 2^-j, j = 0..2K, top = min(2^K tau_prev, tau_max),
 *    tau_max = cap h / max|d|; the largest passing step is taken; if none passes the ladder
 *    moves 2K+1 halvings down; below tau_min_rel * tau_max the level stops;
 *  - stopping: E_k - E_{k+1} < eps, or iter_max accepted steps, or a failed line search, or
 *    G.d <= 0;
 *  - scans: the serial, Brent-Kung, Kogge-Stone and Sklansky listings in their standard
 *    0-based forms for any element count (the Kogge-Stone inner loop starts at 2^i); the
 *    distributed chapter's general strategy with its global scan taken inclusive in place
 *    (Brent-Kung over the chunk ends), so each chunk end is final after the global stage and
 *    local stage two touches the other elements only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int levels;          /* number of grid levels m1 - m0 + 1 */
  double lambda;       /* Dirichlet weight */
  double beta;         /* smoother width in cells */
  double sigma;        /* Armijo constant */
  int ladder_k;        /* K: 2K+1 step sizes per line-search pass */
  double cap;          /* largest step, in cells of the current level */
  double tau_min_rel;  /* line search gives up below tau_min_rel * tau_max */
  double eps;          /* energy-decrease stopping threshold */
  int iter_max;        /* accepted steps per level */
} or_params;

#define OR_MAX_LEVELS 16
typedef struct {
  int iters[OR_MAX_LEVELS];   /* accepted steps per level, index 0 = coarsest */
  int trials[OR_MAX_LEVELS];  /* line-search passes per level */
  double energy;              /* final energy at the finest level */
  double ncc;                 /* final NCC at the finest level */
  int flags;                  /* OR_FLAG_* */
  double tie_gap;             /* with replayed stopping decisions: the largest distance by which
                                 the energy test would have decided a replayed step the other way
                                 (0 when every replayed decision agrees with the test) */
  double armijo_gap;          /* with replayed line-search decisions: the same for the Armijo test
                                 (a larger step it would accept, or the replayed step it would
                                 reject) */
} or_stats;

/* Test switch: decisions another implementation took, replayed in place of the oracle's own
   tests so that two implementations can be compared along one decision sequence where rounding
   decides near-ties differently. force[l - m0] (or -1) is the number of accepted steps of level
   l; rungs[k] is the ladder position J of the k-th accepted step of the registration (levels in
   order, coarsest first): the step top 2^-J of that iteration's ladder. The oracle still
   evaluates its own tests and records in stop_gap / armijo_gap how far they are from each
   replayed decision. */
typedef struct {
  const int* force;
  const unsigned char* rungs;
  int cap;   /* entries in rungs */
  int pos;   /* next entry of rungs */
  double stop_gap, armijo_gap;
} replay_t;

enum { OR_FLAG_NONCONV = 1, OR_FLAG_NAN = 2 };
#define OR_TRACE_W 8

/* ----------------------------------------------------------------------------------------- */
/* Restriction and prolongation (Multilevel section)                                           */

static double fw_weight(int p) { return p == 0 ? 2.0 : 1.0; }

/* Full weighting 1/16 [1 2 1; 2 4 2; 1 2 1]; coarse node (A, B) sits on fine node (2A, 2B). */
void or_restrict(const double* f, int nf, double* g) {
  int nc = (nf - 1) / 2 + 1;
  for (int A = 0; A < nc; ++A)
    for (int B = 0; B < nc; ++B) {
      double s = 0.0, w = 0.0;
      for (int p = -1; p <= 1; ++p)
        for (int q = -1; q <= 1; ++q) {
          int a = 2 * A + p, b = 2 * B + q;
          if (a < 0 || a >= nf || b < 0 || b >= nf) continue;
          double wt = fw_weight(p) * fw_weight(q);
          s += wt * f[a * nf + b];
          w += wt;
        }
      g[A * nc + B] = s / w;
    }
}

/* Bilinear prolongation: copy coarse nodes, average 2 neighbours on edges, 4 on cell centres. */
void or_prolong(const double* c, int nc, double* f) {
  int nf = 2 * (nc - 1) + 1;
  for (int a = 0; a < nf; ++a)
    for (int b = 0; b < nf; ++b) {
      int A = a / 2, B = b / 2;
      double v;
      if (a % 2 == 0 && b % 2 == 0) v = c[A * nc + B];
      else if (a % 2 == 0) v = 0.5 * (c[A * nc + B] + c[A * nc + B + 1]);
      else if (b % 2 == 0) v = 0.5 * (c[A * nc + B] + c[(A + 1) * nc + B]);
      else v = 0.25 * (c[A * nc + B] + c[A * nc + B + 1] + c[(A + 1) * nc + B] +
                       c[(A + 1) * nc + B + 1]);
      f[a * nf + b] = v;
    }
}

/* ----------------------------------------------------------------------------------------- */
/* Clamped bilinear evaluation of a nodal function and its gradient at a point (domain units). */

double or_bilinear(const double* g, int n, double px, double py, double* gx, double* gy) {
  double h = 1.0 / (n - 1);
  double s = px / h, t = py / h;
  int outx = (s < 0.0 || s > n - 1), outy = (t < 0.0 || t > n - 1);
  if (s < 0.0) s = 0.0;
  if (s > n - 1) s = n - 1;
  if (t < 0.0) t = 0.0;
  if (t > n - 1) t = n - 1;
  int b0 = (int)floor(s), a0 = (int)floor(t);
  if (b0 > n - 2) b0 = n - 2;
  if (a0 > n - 2) a0 = n - 2;
  double fx = s - b0, fy = t - a0;
  double v00 = g[a0 * n + b0], v01 = g[a0 * n + b0 + 1];
  double v10 = g[(a0 + 1) * n + b0], v11 = g[(a0 + 1) * n + b0 + 1];
  if (gx) *gx = outx ? 0.0 : ((1.0 - fy) * (v01 - v00) + fy * (v11 - v10)) / h;
  if (gy) *gy = outy ? 0.0 : ((1.0 - fx) * (v10 - v00) + fx * (v11 - v01)) / h;
  return (1.0 - fy) * ((1.0 - fx) * v00 + fx * v01) + fy * ((1.0 - fx) * v10 + fx * v11);
}

/* ----------------------------------------------------------------------------------------- */
/* FE matrices (Spatial discretization section).                                              */
/* A symmetric tridiagonal 1-D matrix with end diagonal de, interior diagonal di, off-diagonal  */
/* o, applied along one axis of a 2-D nodal array (axis 0: along x within rows; 1: along y).    */

static void tri_apply(const double* f, double* g, int n, int axis, double de, double di,
                      double o) {
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      int i = axis == 0 ? b : a;
      int st = axis == 0 ? 1 : n;
      int idx = a * n + b;
      double d = (i == 0 || i == n - 1) ? de : di;
      double v = d * f[idx];
      if (i > 0) v += o * f[idx - st];
      if (i < n - 1) v += o * f[idx + st];
      g[idx] = v;
    }
}

/* 1-D P1 mass matrix M1 = (h/6) tridiag(1, [2 4 ... 4 2], 1). */
static void m1_apply(const double* f, double* g, int n, int axis) {
  double h = 1.0 / (n - 1);
  tri_apply(f, g, n, axis, h / 3.0, 2.0 * h / 3.0, h / 6.0);
}
/* 1-D P1 stiffness matrix K1 = (1/h) tridiag(-1, [1 2 ... 2 1], -1). */
static void k1_apply(const double* f, double* g, int n, int axis) {
  double h = 1.0 / (n - 1);
  tri_apply(f, g, n, axis, 1.0 / h, 2.0 / h, -1.0 / h);
}

/* M F with M = M1 (x) M1 (bilinear mass matrix). */
void or_mass_apply(const double* f, int n, double* out) {
  double* t = malloc(sizeof(double) * n * n);
  m1_apply(f, t, n, 0);
  m1_apply(t, out, n, 1);
  free(t);
}

/* K F with K = K1 (x) M1 + M1 (x) K1 (bilinear stiffness matrix, int |grad f|^2 = F^T K F). */
void or_stiff_apply(const double* f, int n, double* out) {
  size_t nn = (size_t)n * n;
  double* t1 = malloc(sizeof(double) * nn);
  double* t2 = malloc(sizeof(double) * nn);
  m1_apply(f, t1, n, 0);
  k1_apply(t1, out, n, 1);  /* derivative across rows (y), mass along x */
  k1_apply(f, t1, n, 0);
  m1_apply(t1, t2, n, 1);   /* derivative along x, mass across rows */
  for (size_t i = 0; i < nn; ++i) out[i] += t2[i];
  free(t1);
  free(t2);
}

static double dot(const double* a, const double* b, size_t n) {
  double s = 0.0;
  for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Mean 1^T M F and standard deviation sqrt(F_c^T M F_c), F_c = F - mean (|Omega| = 1).
   Writes the normalised F~ = F_c / sigma when out != NULL and sigma > 0.
   Returns -1 if sigma == 0 (sigma <= 1e-12 max(1, |mean|) counts as 0). */
int or_normalize(const double* f, int n, double* out, double* mean, double* sigma) {
  size_t nn = (size_t)n * n;
  double* mf = malloc(sizeof(double) * nn);
  double* fc = malloc(sizeof(double) * nn);
  or_mass_apply(f, n, mf);
  double m = 0.0;
  for (size_t i = 0; i < nn; ++i) m += mf[i];  /* 1^T M F */
  for (size_t i = 0; i < nn; ++i) fc[i] = f[i] - m;
  or_mass_apply(fc, n, mf);
  double var = dot(fc, mf, nn);
  double s = var > 0.0 ? sqrt(var) : 0.0;
  /* a frame counts as constant when sigma is at rounding level relative to its mean */
  if (s <= 1e-12 * fmax(1.0, fabs(m))) s = 0.0;
  if (mean) *mean = m;
  if (sigma) *sigma = s;
  if (out && s > 0.0)
    for (size_t i = 0; i < nn; ++i) out[i] = fc[i] / s;
  free(mf);
  free(fc);
  return s > 0.0 ? 0 : -1;
}

/* ----------------------------------------------------------------------------------------- */
/* Energy and gradient (NCC + Dirichlet energy, E[phi] and its first variation).               */
/* The similarity integrals are evaluated with the 2x2 Gauss rule on every element, the rule   */
/* that integrates the Q1 mass matrix exactly (so for Q1 integrands they equal the F^T M G     */
/* forms). The template is composed with phi at the quadrature points:                          */
/*   q = element point, u(q) = sum_corners psi(q) u_corner, T_phi(q) = T(q + u(q)),             */
/*   mean = sum_q w T_phi(q), sigma^2 = sum_q w (T_phi(q) - mean)^2,                            */
/*   NCC = sum_q w R~(q) (T_phi(q) - mean) / sigma, w = h^2 / 4.                                 */

typedef struct {
  int n;
  const double* Rn;  /* normalised reference R~ (nodal) */
  const double* T;   /* template (nodal) */
} level_data;

static const double GP[2] = {0.21132486540518711775, 0.78867513459481288225};  /* (1 -+ 1/sqrt3)/2 */

/* Quadrature point (element (a, b), local point (p, q)) -> flat index. */
static size_t qidx(int n, int a, int b, int p, int q) {
  return ((((size_t)a * (n - 1) + b) * 2 + p) * 2 + q);
}

/* Bilinear basis weights of the 4 element corners at local point (xi, eta):
   corners ordered (a,b), (a,b+1), (a+1,b), (a+1,b+1). */
static void basis(double xi, double eta, double psi[4]) {
  psi[0] = (1.0 - xi) * (1.0 - eta);
  psi[1] = xi * (1.0 - eta);
  psi[2] = (1.0 - xi) * eta;
  psi[3] = xi * eta;
}

/* Sample T_phi, its gradient and R~ at every quadrature point. */
static void warp_q(const level_data* L, const double* u, double* Tq, double* dTx, double* dTy,
                   double* Rq) {
  int n = L->n;
  double h = 1.0 / (n - 1);
  size_t nn = (size_t)n * n;
  for (int a = 0; a < n - 1; ++a)
    for (int b = 0; b < n - 1; ++b) {
      size_t c[4] = {(size_t)a * n + b, (size_t)a * n + b + 1, (size_t)(a + 1) * n + b,
                     (size_t)(a + 1) * n + b + 1};
      for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) {
          double psi[4];
          basis(GP[q], GP[p], psi);
          double ux = 0.0, uy = 0.0, r = 0.0;
          for (int k = 0; k < 4; ++k) {
            ux += psi[k] * u[c[k]];
            uy += psi[k] * u[nn + c[k]];
            r += psi[k] * L->Rn[c[k]];
          }
          double px = (b + GP[q]) * h + ux, py = (a + GP[p]) * h + uy;
          double gx, gy;
          size_t qi = qidx(n, a, b, p, q);
          Tq[qi] = or_bilinear(L->T, n, px, py, &gx, &gy);
          if (dTx) dTx[qi] = gx;
          if (dTy) dTy[qi] = gy;
          if (Rq) Rq[qi] = r;
        }
    }
}

/* Mean, sigma and NCC of the sampled template against R~ (all by the quadrature rule).
   Returns sigma (0 when the warped template is constant; NCC is then 0). */
static double ncc_q(int n, const double* Tq, const double* Rq, double* mean, double* ncc) {
  double h = 1.0 / (n - 1);
  double w = h * h / 4.0;
  size_t nq = (size_t)4 * (n - 1) * (n - 1);
  double m = 0.0;
  for (size_t i = 0; i < nq; ++i) m += w * Tq[i];
  double var = 0.0;
  for (size_t i = 0; i < nq; ++i) var += w * (Tq[i] - m) * (Tq[i] - m);
  double s = var > 0.0 ? sqrt(var) : 0.0;
  double c = 0.0;
  if (s > 0.0)
    for (size_t i = 0; i < nq; ++i) c += w * Rq[i] * (Tq[i] - m) / s;
  *mean = m;
  *ncc = c;
  return s;
}

static double regulariser(const double* u, int n) {
  size_t nn = (size_t)n * n;
  double* Ku = malloc(sizeof(double) * nn);
  double reg = 0.0;
  for (int c = 0; c < 2; ++c) {
    or_stiff_apply(u + c * nn, n, Ku);
    reg += dot(u + c * nn, Ku, nn);
  }
  free(Ku);
  return reg;
}

/* E(u) = -NCC[R, T o phi] + (lambda/2) sum_c u_c^T K u_c. */
static double energy_level(const level_data* L, const double* u, double lambda, double* ncc_out) {
  int n = L->n;
  size_t nq = (size_t)4 * (n - 1) * (n - 1);
  double* Tq = malloc(sizeof(double) * nq);
  double* Rq = malloc(sizeof(double) * nq);
  warp_q(L, u, Tq, NULL, NULL, Rq);
  double m, ncc;
  ncc_q(n, Tq, Rq, &m, &ncc);
  free(Tq);
  free(Rq);
  if (ncc_out) *ncc_out = ncc;
  return -ncc + 0.5 * lambda * regulariser(u, n);
}

/* dE/du_i = -sum_q w (R~(q) - NCC T~_phi(q)) / sigma * grad T(q + u(q)) psi_i(q)
             + lambda (K u)_i, summed over the quadrature points of the elements around i. */
static void gradient_level(const level_data* L, const double* u, double lambda, double* G) {
  int n = L->n;
  double h = 1.0 / (n - 1);
  double w = h * h / 4.0;
  size_t nn = (size_t)n * n;
  size_t nq = (size_t)4 * (n - 1) * (n - 1);
  double* Tq = malloc(sizeof(double) * nq);
  double* dTx = malloc(sizeof(double) * nq);
  double* dTy = malloc(sizeof(double) * nq);
  double* Rq = malloc(sizeof(double) * nq);
  double* Ku = malloc(sizeof(double) * nn);
  warp_q(L, u, Tq, dTx, dTy, Rq);
  double m, ncc;
  double s = ncc_q(n, Tq, Rq, &m, &ncc);
  memset(G, 0, sizeof(double) * 2 * nn);
  if (s > 0.0) {
    for (int a = 0; a < n - 1; ++a)
      for (int b = 0; b < n - 1; ++b) {
        size_t c[4] = {(size_t)a * n + b, (size_t)a * n + b + 1, (size_t)(a + 1) * n + b,
                       (size_t)(a + 1) * n + b + 1};
        for (int p = 0; p < 2; ++p)
          for (int q = 0; q < 2; ++q) {
            size_t qi = qidx(n, a, b, p, q);
            double f = -w * (Rq[qi] - ncc * (Tq[qi] - m) / s) / s;  /* d(-NCC)/dT_phi(q) */
            double psi[4];
            basis(GP[q], GP[p], psi);
            for (int k = 0; k < 4; ++k) {
              G[c[k]] += f * dTx[qi] * psi[k];
              G[nn + c[k]] += f * dTy[qi] * psi[k];
            }
          }
      }
  }
  for (int cc = 0; cc < 2; ++cc) {
    or_stiff_apply(u + cc * nn, n, Ku);
    for (size_t i = 0; i < nn; ++i) G[cc * nn + i] += lambda * Ku[i];
  }
  free(Tq);
  free(dTx);
  free(dTy);
  free(Rq);
  free(Ku);
}

/* ----------------------------------------------------------------------------------------- */
/* Metric of the gradient flow: d = A^{-1} G, A = S1 (x) S1, S1 = M1 + (beta h)^2 K1.          */

/* Thomas algorithm for a symmetric tridiagonal system along one line of a 2-D array. */
static void thomas_line(double* x, int n, size_t stride, double de, double di, double o,
                        double* cp, double* dp) {
  for (int i = 0; i < n; ++i) {
    double d = (i == 0 || i == n - 1) ? de : di;
    double rhs = x[i * stride];
    if (i == 0) {
      cp[0] = o / d;
      dp[0] = rhs / d;
    } else {
      double den = d - o * cp[i - 1];
      cp[i] = o / den;
      dp[i] = (rhs - o * dp[i - 1]) / den;
    }
  }
  x[(n - 1) * stride] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i) x[i * stride] = dp[i] - cp[i] * x[(i + 1) * stride];
}

void or_smooth(const double* g, int n, double beta, double* out) {
  double h = 1.0 / (n - 1);
  double c = beta * beta * h * h;
  double de = h / 3.0 + c / h, di = 2.0 * h / 3.0 + 2.0 * c / h, o = h / 6.0 - c / h;
  double* cp = malloc(sizeof(double) * n);
  double* dp = malloc(sizeof(double) * n);
  memcpy(out, g, sizeof(double) * n * n);
  for (int b = 0; b < n; ++b) thomas_line(out + b, n, n, de, di, o, cp, dp);  /* along y */
  for (int a = 0; a < n; ++a) thomas_line(out + (size_t)a * n, n, 1, de, di, o, cp, dp); /* x */
  free(cp);
  free(dp);
}

/* ----------------------------------------------------------------------------------------- */
/* Public energy / gradient on raw frames (normalises the reference itself).                  */

double or_energy(const double* R, const double* T, int n, const double* u, double lambda,
                 double* ncc) {
  size_t nn = (size_t)n * n;
  double* Rn = malloc(sizeof(double) * nn);
  if (or_normalize(R, n, Rn, NULL, NULL) != 0) {
    free(Rn);
    return NAN;
  }
  level_data L = {n, Rn, T};
  double e = energy_level(&L, u, lambda, ncc);
  free(Rn);
  return e;
}

int or_gradient(const double* R, const double* T, int n, const double* u, double lambda,
                double* G) {
  size_t nn = (size_t)n * n;
  double* Rn = malloc(sizeof(double) * nn);
  if (or_normalize(R, n, Rn, NULL, NULL) != 0) {
    free(Rn);
    return -1;
  }
  level_data L = {n, Rn, T};
  gradient_level(&L, u, lambda, G);
  free(Rn);
  return 0;
}

/* ----------------------------------------------------------------------------------------- */
/* Gradient flow on one level: forward Euler steps u <- u - tau A^{-1} E'(u) with the Armijo  */
/* ladder described in the header. Returns the number of accepted steps; writes trace records  */
/* [level, step, tau, E_before, E_after, G.d, tau_max, passes] when trace != NULL.             */

/* Test switch: round u to FP32 after every accepted step (off by default). It measures how
   far FP32 storage of the displacement alone moves the result, which bounds the agreement any
   FP32 implementation can reach with this FP64 oracle. */
static int g_u_storage_f32 = 0;
void or_set_u_storage_f32(int on) { g_u_storage_f32 = on != 0; }

typedef struct {
  double* buf;
  int cap;
  int len;
} trace_t;

static void trace_put(trace_t* tr, int level, int step, double tau, double e0, double e1,
                      double gtd, double tmax, int passes) {
  if (!tr || !tr->buf || tr->len >= tr->cap) return;
  double* r = tr->buf + (size_t)tr->len * OR_TRACE_W;
  r[0] = level;
  r[1] = step;
  r[2] = tau;
  r[3] = e0;
  r[4] = e1;
  r[5] = gtd;
  r[6] = tmax;
  r[7] = passes;
  tr->len++;
}

/* force >= 0 (replay_t): the level takes exactly `force` accepted steps (unless the line
   search fails or the flow is stationary first) and the energy-decrease test is not applied;
   -1 is the method itself. rp (may be NULL) supplies replayed ladder positions and collects
   the gaps. */
static int gradient_flow(const level_data* L, double* u, const or_params* p, int level,
                         int force, replay_t* rp, int* trials, int* flags, double* e_out,
                         double* ncc_out, trace_t* tr) {
  int n = L->n;
  size_t nn = (size_t)n * n;
  double h = 1.0 / (n - 1);
  double* G = malloc(sizeof(double) * 2 * nn);
  double* d = malloc(sizeof(double) * 2 * nn);
  double* ut = malloc(sizeof(double) * 2 * nn);
  int K = p->ladder_k;
  double ncc;
  double E = energy_level(L, u, p->lambda, &ncc);
  double tau_prev = INFINITY;
  int steps = 0, passes_total = 0;
  if (!isfinite(E)) *flags |= OR_FLAG_NAN;
  while (isfinite(E) && steps < p->iter_max) {
    gradient_level(L, u, p->lambda, G);
    or_smooth(G, n, p->beta, d);
    or_smooth(G + nn, n, p->beta, d + nn);
    double gtd = dot(G, d, 2 * nn);
    double dmax = 0.0;
    for (size_t i = 0; i < 2 * nn; ++i) dmax = fmax(dmax, fabs(d[i]));
    if (!(gtd > 0.0) || !(dmax > 0.0)) break;           /* stationary */
    double tau_max = p->cap * h / dmax;
    double top = fmin(ldexp(tau_prev, K), tau_max);
    double tau_acc = 0.0, e_acc = E, ncc_acc = ncc;
    int passes = 0;
    if (rp && rp->rungs && rp->pos < rp->cap) {
      /* replayed: rung J of this iteration's ladder; the rungs above it are evaluated with the
         Armijo test only to measure how far it is from the replayed choice */
      int J = rp->rungs[rp->pos++];
      for (int j = 0; j <= J; ++j) {
        double tau = ldexp(top, -j);
        for (size_t i = 0; i < 2 * nn; ++i) ut[i] = u[i] - tau * d[i];
        double nc;
        double e = energy_level(L, ut, p->lambda, &nc);
        double bound = E - p->sigma * tau * gtd;
        if (j < J && e <= bound) rp->armijo_gap = fmax(rp->armijo_gap, bound - e);
        if (j == J) {
          if (e > bound) rp->armijo_gap = fmax(rp->armijo_gap, e - bound);
          tau_acc = tau;
          e_acc = e;
          ncc_acc = nc;
        }
      }
      passes = J / (2 * K + 1) + 1;
    } else {
      while (top >= p->tau_min_rel * tau_max) {
        passes++;
        for (int j = 0; j <= 2 * K; ++j) {                /* largest step first */
          double tau = ldexp(top, -j);
          for (size_t i = 0; i < 2 * nn; ++i) ut[i] = u[i] - tau * d[i];
          double nc;
          double e = energy_level(L, ut, p->lambda, &nc);
          if (e <= E - p->sigma * tau * gtd) {            /* Armijo, sufficient decrease */
            tau_acc = tau;
            e_acc = e;
            ncc_acc = nc;
            break;
          }
        }
        if (tau_acc > 0.0) break;
        top = ldexp(top, -(2 * K + 1));
      }
    }
    passes_total += passes;
    trace_put(tr, level, steps, tau_acc, E, e_acc, gtd, tau_max, passes);
    if (tau_acc == 0.0) break;                            /* line search exhausted */
    for (size_t i = 0; i < 2 * nn; ++i) u[i] -= tau_acc * d[i];
    if (g_u_storage_f32)
      for (size_t i = 0; i < 2 * nn; ++i) u[i] = (double)(float)u[i];
    double dec = E - e_acc;
    E = e_acc;
    ncc = ncc_acc;
    tau_prev = tau_acc;
    steps++;
    if (force >= 0 && rp) { /* how far the energy test is from the replayed decision */
      if (steps < force) rp->stop_gap = fmax(rp->stop_gap, p->eps - dec);
      else if (steps < p->iter_max) rp->stop_gap = fmax(rp->stop_gap, dec - p->eps);
    }
    if (force >= 0 ? steps >= force : dec < p->eps) break; /* converged (or replayed stop) */
    if (steps >= p->iter_max) *flags |= OR_FLAG_NONCONV;
  }
  if (trials) *trials = passes_total;
  if (e_out) *e_out = E;
  if (ncc_out) *ncc_out = ncc;
  free(G);
  free(d);
  free(ut);
  return steps;
}

/* One level of gradient flow on raw frames (normalises the reference). */
int or_gradient_flow(const double* R, const double* T, int n, double* u, const or_params* p,
                     int* steps, int* passes, double* energy, double* trace, int trace_cap,
                     int* trace_len) {
  size_t nn = (size_t)n * n;
  double* Rn = malloc(sizeof(double) * nn);
  if (or_normalize(R, n, Rn, NULL, NULL) != 0) {
    free(Rn);
    return -1;
  }
  level_data L = {n, Rn, T};
  trace_t tr = {trace, trace_cap, 0};
  int flags = 0;
  int s = gradient_flow(&L, u, p, 0, -1, NULL, passes, &flags, energy, NULL, &tr);
  if (steps) *steps = s;
  if (trace_len) *trace_len = tr.len;
  free(Rn);
  return flags;
}

/* ----------------------------------------------------------------------------------------- */
/* Function A: multilevel gradient flow (Algorithm "multigrid_gradient").                      */
/* R, T are finest-level nodal frames (nf = 2^L + 1); u0 (finest, domain units) may be NULL    */
/* for the identity; u_out receives the finest-level displacement. Returns 0, or -1 when the  */
/* reference is constant on some level, or -2 on bad sizes.                                     */

static int log2_exact(int m) {
  int l = 0;
  while ((1 << l) < m) ++l;
  return (1 << l) == m ? l : -1;
}

/* Levels m0..L of the pyramid of R and T: raw restrictions, then the normalised reference
   (zero mean, unit standard deviation). Returns -1 when the reference is constant on a level. */
typedef struct {
  double* Rl[OR_MAX_LEVELS + 1];
  double* Tl[OR_MAX_LEVELS + 1];
  double* Rn[OR_MAX_LEVELS + 1];
  int m0, L;
} pyramid_t;

static int pyramid_build(pyramid_t* py, const double* R, const double* T, int L, int m0) {
  int rc = 0;
  py->m0 = m0;
  py->L = L;
  for (int l = L; l >= m0; --l) {
    int n = (1 << l) + 1;
    size_t nn = (size_t)n * n;
    py->Rl[l] = malloc(sizeof(double) * nn);
    py->Tl[l] = malloc(sizeof(double) * nn);
    py->Rn[l] = malloc(sizeof(double) * nn);
    if (l == L) {
      memcpy(py->Rl[l], R, sizeof(double) * nn);
      memcpy(py->Tl[l], T, sizeof(double) * nn);
    } else {
      or_restrict(py->Rl[l + 1], (1 << (l + 1)) + 1, py->Rl[l]);
      or_restrict(py->Tl[l + 1], (1 << (l + 1)) + 1, py->Tl[l]);
    }
    if (or_normalize(py->Rl[l], n, py->Rn[l], NULL, NULL) != 0) rc = -1;
  }
  return rc;
}

static void pyramid_free(pyramid_t* py) {
  for (int l = py->L; l >= py->m0; --l) {
    free(py->Rl[l]);
    free(py->Tl[l]);
    free(py->Rn[l]);
  }
}

/* Gradient flow on levels start..L from the guess u (level `start`, owned: freed here), each
   result prolongated as the next level's start. Statistics are indexed from level m0. */
static void run_levels(const pyramid_t* py, int start, double* u, const or_params* p,
                       replay_t* rp, double* u_out, or_stats* st, double* trace,
                       int trace_cap, int* trace_len) {
  int L = py->L, m0 = py->m0, nf = (1 << L) + 1;
  trace_t tr = {trace, trace_cap, 0};
  if (st) memset(st, 0, sizeof(*st));
  int flags = 0;
  double e = 0.0, ncc = 0.0;
  for (int l = start; l <= L; ++l) {
    int n = (1 << l) + 1;
    level_data LD = {n, py->Rn[l], py->Tl[l]};
    int passes = 0;
    int force = rp && rp->force ? rp->force[l - m0] : -1;
    int steps = gradient_flow(&LD, u, p, l, force, rp, &passes, &flags, &e, &ncc, &tr);
    if (st) {
      st->iters[l - m0] = steps;
      st->trials[l - m0] = passes;
    }
    if (l < L) {
      int nn2 = (1 << (l + 1)) + 1;
      double* uf = malloc(sizeof(double) * 2 * nn2 * nn2);
      for (int c = 0; c < 2; ++c)
        or_prolong(u + (size_t)c * n * n, n, uf + (size_t)c * nn2 * nn2);
      free(u);
      u = uf;
    }
  }
  memcpy(u_out, u, sizeof(double) * 2 * nf * nf);
  free(u);
  if (st) {
    st->energy = e;
    st->ncc = ncc;
    st->flags = flags;
    st->tie_gap = rp ? rp->stop_gap : 0.0;
    st->armijo_gap = rp ? rp->armijo_gap : 0.0;
  }
  if (trace_len) *trace_len = tr.len;
}

/* force (may be NULL): per level from m0, the number of accepted steps to take instead of
   applying the energy-decrease stopping test (-1: the test applies); rungs (may be NULL,
   rung_cap entries): the ladder position of every accepted step (replay_t). */
int or_register_f(const double* R, const double* T, int nf, const double* u0,
                  const or_params* p, const int* force, const unsigned char* rungs,
                  int rung_cap, double* u_out, or_stats* st, double* trace, int trace_cap,
                  int* trace_len) {
  replay_t rp = {force, rungs, rungs ? rung_cap : 0, 0, 0.0, 0.0};
  int L = log2_exact(nf - 1);
  if (L < 1 || p->levels < 1 || p->levels > L || p->levels > OR_MAX_LEVELS) return -2;
  int m0 = L - p->levels + 1;
  pyramid_t py;
  int rc = pyramid_build(&py, R, T, L, m0);
  if (rc == 0) {
    /* Initial guess on the coarsest level: restrict u0 down to m0 (identity if NULL). */
    int n0 = (1 << m0) + 1;
    double* u = calloc((size_t)2 * n0 * n0, sizeof(double));
    if (u0) {
      int n = nf;
      double* cur = malloc(sizeof(double) * 2 * nf * nf);
      memcpy(cur, u0, sizeof(double) * 2 * nf * nf);
      for (int l = L; l > m0; --l) {
        int nc = (1 << (l - 1)) + 1;
        double* nxt = malloc(sizeof(double) * 2 * nc * nc);
        for (int c = 0; c < 2; ++c)
          or_restrict(cur + (size_t)c * n * n, n, nxt + (size_t)c * nc * nc);
        free(cur);
        cur = nxt;
        n = nc;
      }
      memcpy(u, cur, sizeof(double) * 2 * n0 * n0);
      free(cur);
    }
    run_levels(&py, m0, u, p, (force || rungs) ? &rp : NULL, u_out, st, trace, trace_cap,
               trace_len);
  }
  pyramid_free(&py);
  return rc;
}

int or_register(const double* R, const double* T, int nf, const double* u0, const or_params* p,
                double* u_out, or_stats* st, double* trace, int trace_cap, int* trace_len) {
  return or_register_f(R, T, nf, u0, p, NULL, NULL, 0, u_out, st, trace, trace_cap, trace_len);
}

/* Function A started on level `start` (m0 <= start <= L) from the guess u_start given on that
   level ([2][n_start][n_start], domain units): the coarser levels are skipped, as a warm start
   from a predicted displacement does. The reference is still checked on levels m0..L. */
int or_register_from(const double* R, const double* T, int nf, int start,
                     const double* u_start, const or_params* p, double* u_out, or_stats* st,
                     double* trace, int trace_cap, int* trace_len) {
  int L = log2_exact(nf - 1);
  if (L < 1 || p->levels < 1 || p->levels > L || p->levels > OR_MAX_LEVELS) return -2;
  int m0 = L - p->levels + 1;
  if (start < m0 || start > L || !u_start) return -2;
  pyramid_t py;
  int rc = pyramid_build(&py, R, T, L, m0);
  if (rc == 0) {
    int ns = (1 << start) + 1;
    double* u = malloc(sizeof(double) * 2 * ns * ns);
    memcpy(u, u_start, sizeof(double) * 2 * ns * ns);
    run_levels(&py, start, u, p, NULL, u_out, st, trace, trace_cap, trace_len);
  }
  pyramid_free(&py);
  return rc;
}

/* ----------------------------------------------------------------------------------------- */
/* Rigid variant (definition of a rigid transformation): phi(x) = R(alpha) x + t, parameters  */
/* p = (alpha, t0, t1) in domain units, rotation about the domain origin as printed. Its     */
/* nodal displacement u_p(x_i) = phi(x_i) - x_i is affine, which bilinear interpolation       */
/* reproduces exactly, so the energy is the field energy of u_p with lambda = 0 (-NCC: a rigid */
/* motion has no regulariser) and the parameter gradient is the chain rule through the nodes: */
/* dE/dp_k = sum_i G_i . psi_k(x_i), G the nodal gradient at lambda = 0, psi_alpha =          */
/* R'(alpha) x, psi_t0 = (1, 0), psi_t1 = (0, 1). Steepest descent in p (Euclidean metric)    */
/* with the Armijo ladder, tau_max from the largest nodal |d| of the direction's field, and   */
/* the stopping rules of the field flow; the multilevel loop carries p from level to level.   */

static void rigid_field(int n, const double p[3], double* u) {
  size_t nn = (size_t)n * n;
  double h = 1.0 / (n - 1), c = cos(p[0]), s = sin(p[0]);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double x = b * h, y = a * h;
      size_t i = (size_t)a * n + b;
      u[i] = c * x - s * y + p[1] - x;
      u[nn + i] = s * x + c * y + p[2] - y;
    }
}

static int rigid_flow(const level_data* L, double p[3], const or_params* pr, int force,
                      replay_t* rp, int* passes_out, int* flags, double* e_out,
                      double* ncc_out) {
  int n = L->n;
  size_t nn = (size_t)n * n;
  double h = 1.0 / (n - 1);
  double* u = malloc(sizeof(double) * 2 * nn);
  double* G = malloc(sizeof(double) * 2 * nn);
  int K = pr->ladder_k;
  rigid_field(n, p, u);
  double ncc;
  double E = energy_level(L, u, 0.0, &ncc);
  double tau_prev = INFINITY;
  int steps = 0, passes_total = 0;
  if (!isfinite(E)) *flags |= OR_FLAG_NAN;
  while (isfinite(E) && steps < pr->iter_max) {
    gradient_level(L, u, 0.0, G);
    double c = cos(p[0]), s = sin(p[0]);
    double g[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double x = b * h, y = a * h;
        size_t i = (size_t)a * n + b;
        g[0] += G[i] * (-s * x - c * y) + G[nn + i] * (c * x - s * y);
        g[1] += G[i];
        g[2] += G[nn + i];
      }
    double d[3] = {g[0], g[1], g[2]};
    double gtd = d[0] * g[0] + d[1] * g[1] + d[2] * g[2];
    double dmax = 0.0;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double x = b * h, y = a * h;
        dmax = fmax(dmax, fabs(d[0] * (-s * x - c * y) + d[1]));
        dmax = fmax(dmax, fabs(d[0] * (c * x - s * y) + d[2]));
      }
    if (!(gtd > 0.0) || !(dmax > 0.0)) break;
    double tau_max = pr->cap * h / dmax;
    double top = fmin(ldexp(tau_prev, K), tau_max);
    double tau_acc = 0.0, e_acc = E, ncc_acc = ncc;
    double pt[3];
    if (rp && rp->rungs && rp->pos < rp->cap) {  /* replayed rung (see gradient_flow) */
      int J = rp->rungs[rp->pos++];
      for (int j = 0; j <= J; ++j) {
        double tau = ldexp(top, -j);
        for (int k = 0; k < 3; ++k) pt[k] = p[k] - tau * d[k];
        rigid_field(n, pt, u);
        double nc;
        double e = energy_level(L, u, 0.0, &nc);
        double bound = E - pr->sigma * tau * gtd;
        if (j < J && e <= bound) rp->armijo_gap = fmax(rp->armijo_gap, bound - e);
        if (j == J) {
          if (e > bound) rp->armijo_gap = fmax(rp->armijo_gap, e - bound);
          tau_acc = tau;
          e_acc = e;
          ncc_acc = nc;
        }
      }
      passes_total += J / (2 * K + 1) + 1;
    } else {
      while (top >= pr->tau_min_rel * tau_max) {
        passes_total++;
        for (int j = 0; j <= 2 * K; ++j) {
          double tau = ldexp(top, -j);
          for (int k = 0; k < 3; ++k) pt[k] = p[k] - tau * d[k];
          rigid_field(n, pt, u);
          double nc;
          double e = energy_level(L, u, 0.0, &nc);
          if (e <= E - pr->sigma * tau * gtd) {
            tau_acc = tau;
            e_acc = e;
            ncc_acc = nc;
            break;
          }
        }
        if (tau_acc > 0.0) break;
        top = ldexp(top, -(2 * K + 1));
      }
    }
    if (tau_acc == 0.0) break;
    for (int k = 0; k < 3; ++k) p[k] -= tau_acc * d[k];
    rigid_field(n, p, u);
    double dec = E - e_acc;
    E = e_acc;
    ncc = ncc_acc;
    tau_prev = tau_acc;
    steps++;
    if (force >= 0 && rp) { /* how far the energy test is from the replayed decision */
      if (steps < force) rp->stop_gap = fmax(rp->stop_gap, pr->eps - dec);
      else if (steps < pr->iter_max) rp->stop_gap = fmax(rp->stop_gap, dec - pr->eps);
    }
    if (force >= 0 ? steps >= force : dec < pr->eps) break;
    if (steps >= pr->iter_max) *flags |= OR_FLAG_NONCONV;
  }
  if (passes_out) *passes_out = passes_total;
  if (e_out) *e_out = E;
  if (ncc_out) *ncc_out = ncc;
  free(u);
  free(G);
  return steps;
}

/* Rigid registration of T to R (nodal frames of side nf) from p_init (NULL: identity) over the
   multilevel pyramid; p_out receives the parameters (domain units). Returns 0, -1 for a constant
   reference, -2 for bad sizes. */
/* force, rungs: as for or_register_f (may be NULL). */
int or_register_rigid_f(const double* R, const double* T, int nf, const double* p_init,
                        const or_params* pr, const int* force, const unsigned char* rungs,
                        int rung_cap, double* p_out, or_stats* st) {
  replay_t rp = {force, rungs, rungs ? rung_cap : 0, 0, 0.0, 0.0};
  int L = log2_exact(nf - 1);
  if (L < 1 || pr->levels < 1 || pr->levels > L || pr->levels > OR_MAX_LEVELS) return -2;
  int m0 = L - pr->levels + 1;
  pyramid_t py;
  int rc = pyramid_build(&py, R, T, L, m0);
  if (rc == 0) {
    double p[3] = {0.0, 0.0, 0.0};
    if (p_init) memcpy(p, p_init, sizeof p);
    if (st) memset(st, 0, sizeof(*st));
    int flags = 0;
    double e = 0.0, ncc = 0.0;
    for (int l = m0; l <= L; ++l) {
      level_data LD = {(1 << l) + 1, py.Rn[l], py.Tl[l]};
      int passes = 0;
      int steps = rigid_flow(&LD, p, pr, force ? force[l - m0] : -1, &rp, &passes, &flags, &e,
                             &ncc);
      if (st) {
        st->iters[l - m0] = steps;
        st->trials[l - m0] = passes;
      }
    }
    memcpy(p_out, p, sizeof p);
    if (st) {
      st->energy = e;
      st->ncc = ncc;
      st->flags = flags;
      st->tie_gap = rp.stop_gap;
      st->armijo_gap = rp.armijo_gap;
    }
  }
  pyramid_free(&py);
  return rc;
}

/* ----------------------------------------------------------------------------------------- */
/* Composition (Registration for series of images): (phi_jk o phi_ij)(x) = phi_jk(phi_ij(x)),  */
/* i.e. w(x) = u_ij(x) + u_jk(x + u_ij(x)), bilinear and clamped. out may alias u_ij.          */

void or_compose(const double* uij, const double* ujk, int n, double* out) {
  double h = 1.0 / (n - 1);
  size_t nn = (size_t)n * n;
  double* w = malloc(sizeof(double) * 2 * nn);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      size_t i = (size_t)a * n + b;
      double px = b * h + uij[i], py = a * h + uij[nn + i];
      w[i] = uij[i] + or_bilinear(ujk, n, px, py, NULL, NULL);
      w[nn + i] = uij[nn + i] + or_bilinear(ujk + nn, n, px, py, NULL, NULL);
    }
  memcpy(out, w, sizeof(double) * 2 * nn);
  free(w);
}

/* ----------------------------------------------------------------------------------------- */
/* Series registration as an inclusive prefix scan with operator B (def. of image series       */
/* registration; eq. of the prefix sum with B).                                                */
/* Elements x_m = (m, m+1, A(f_m, f_{m+1}, id)), m = 0..N-2; y_m = x_0 (.) ... (.) x_m.        */
/* (i, j, u) (.) (j, k, v) = (i, k, A(f_i, f_k, v o u)).                                         */

enum { OR_SCAN_SEQUENTIAL = 0, OR_SCAN_BRENT_KUNG = 1, OR_SCAN_KOGGE_STONE = 2, OR_SCAN_SKLANSKY = 3,
       OR_SCAN_GENERAL = 4, OR_SCAN_BLELLOCH = 5, OR_SCAN_REDUCE_THEN_SCAN = 6 };

typedef struct {
  int i, k;
  double* u;
} elem_t;

typedef struct {
  const double* frames;
  int nf;
  const or_params* p;
  or_stats* op_stats;  /* per op, in execution order; may be NULL */
  int* op_pairs;       /* (i, j, k) per op in execution order; may be NULL */
  const int* force_b;  /* per op, OR_MAX_LEVELS replayed step counts (see or_register_f); or NULL */
  const unsigned char* rungs_b;  /* per op, rung_cap replayed ladder positions; or NULL */
  int rung_cap;
  int n_ops;
  int err;
} series_ctx;

static void apply_b(series_ctx* S, const elem_t* left, elem_t* right, int op_index) {
  size_t nn = (size_t)S->nf * S->nf;
  if (left->k != right->i) {
    S->err = -4;
    return;
  }
  double* w = malloc(sizeof(double) * 2 * nn);
  or_compose(left->u, right->u, S->nf, w);
  or_stats st;
  int rc = or_register_f(S->frames + (size_t)left->i * nn, S->frames + (size_t)right->k * nn,
                         S->nf, w, S->p,
                         S->force_b ? S->force_b + (size_t)op_index * OR_MAX_LEVELS : NULL,
                         S->rungs_b ? S->rungs_b + (size_t)op_index * S->rung_cap : NULL,
                         S->rung_cap, right->u, &st, NULL, 0, NULL);
  if (rc != 0) S->err = rc;
  if (S->op_stats) S->op_stats[op_index] = st;
  if (S->op_pairs) {
    S->op_pairs[3 * op_index] = left->i;
    S->op_pairs[3 * op_index + 1] = left->k;
    S->op_pairs[3 * op_index + 2] = right->k;
  }
  right->i = left->i;
  free(w);
}

/* frames: N finest-level nodal frames; u_out: N x 2 x nf x nf, u_out[0] = 0.
   a_stats: N-1 entries (may be NULL); b_stats / b_pairs: up to 2N entries (may be NULL).
   Returns the number of B ops, or a negative error. */
/* Applies the ops (src[t], dst[t]), t < cnt, of one step (mutually independent) in parallel. */
static void apply_step(series_ctx* S, elem_t* x, const int* src, const int* dst, int cnt,
                       int op0) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < cnt; ++t) apply_b(S, &x[src[t]], &x[dst[t]], op0 + t);
}

/* General strategy of the distributed chapter on `workers` workers (0: ceil(sqrt(M))).
   Worker I owns x[l_I .. r_I]; K = floor(M/P) + 1 elements for the first M mod P workers and
   floor(M/P) for the rest. Local stage one: every worker runs the serial scan on its chunk.
   Global stage: the chunk ends x[r_0], ..., x[r_{P-1}] are scanned with Brent-Kung in place,
   which leaves x[r_{I-1}] = x_0 (.) ... (.) x_{r_{I-1}}, the exclusive value worker I needs, and
   makes x[r_I] final. Local stage two: worker I > 0 combines that value with each of its other
   elements. Returns the number of ops. */
static int scan_general(series_ctx* S, elem_t* x, int M, int workers) {
  int P = workers > 0 ? workers : (int)ceil(sqrt((double)M));
  if (P > M) P = M;
  int* l = malloc(sizeof(int) * P);
  int* r = malloc(sizeof(int) * P);
  int K = M / P, extra = M % P, at = 0, kmax = 0;
  for (int I = 0; I < P; ++I) {
    int k = K + (I < extra ? 1 : 0);
    l[I] = at;
    r[I] = at + k - 1;
    at += k;
    if (k > kmax) kmax = k;
  }
  int* src = malloc(sizeof(int) * (M > 0 ? M : 1));
  int* dst = malloc(sizeof(int) * (M > 0 ? M : 1));
  int ops = 0, cnt;
  /* local stage one: step i of every worker's serial scan, the workers side by side */
  for (int i = 1; i < kmax; ++i) {
    cnt = 0;
    for (int I = 0; I < P; ++I)
      if (l[I] + i <= r[I]) {
        src[cnt] = l[I] + i - 1;
        dst[cnt] = l[I] + i;
        ++cnt;
      }
    apply_step(S, x, src, dst, cnt, ops);
    ops += cnt;
  }
  /* global stage: Brent-Kung over the chunk ends (up-sweep, then down-sweep) */
  for (int d = 1; d < P; d *= 2) {
    cnt = 0;
    for (int j = 2 * d - 1; j < P; j += 2 * d) {
      src[cnt] = r[j - d];
      dst[cnt] = r[j];
      ++cnt;
    }
    apply_step(S, x, src, dst, cnt, ops);
    ops += cnt;
  }
  int dtop = 1;
  while (dtop * 2 < P) dtop *= 2;
  for (int d = dtop; d >= 1; d /= 2) {
    cnt = 0;
    for (int j = 3 * d - 1; j < P; j += 2 * d) {
      src[cnt] = r[j - d];
      dst[cnt] = r[j];
      ++cnt;
    }
    apply_step(S, x, src, dst, cnt, ops);
    ops += cnt;
  }
  /* local stage two: worker I > 0 applies the total before its chunk to its other elements */
  cnt = 0;
  for (int I = 1; I < P; ++I)
    for (int j = l[I]; j < r[I]; ++j) {
      src[cnt] = r[I - 1];
      dst[cnt] = j;
      ++cnt;
    }
  apply_step(S, x, src, dst, cnt, ops);
  ops += cnt;
  free(l);
  free(r);
  free(src);
  free(dst);
  return ops;
}

/* A scan element that may be the identity element of the operator (Blelloch's exclusive scan
   starts from it): id != 0 means the identity, whose combination with any element is that
   element, at no cost. Its buffer u is owned by the element. */
typedef struct {
  int id, i, k;
  double* u;
} velem_t;

/* dst <- left (.) right. With an identity operand the other is copied; otherwise B registers
   frame right.k to frame left.i from the composition of the two fields (op numbered op_index).
   dst may be left or right. */
static void combine(series_ctx* S, const velem_t* left, const velem_t* right, velem_t* dst,
                    int op_index) {
  size_t nn = (size_t)S->nf * S->nf;
  if (left->id || right->id) {
    const velem_t* src = left->id ? right : left;
    if (src != dst) {
      dst->id = src->id;
      dst->i = src->i;
      dst->k = src->k;
      if (!src->id) memcpy(dst->u, src->u, sizeof(double) * 2 * nn);
    }
    return;
  }
  elem_t l = {left->i, left->k, left->u}, r = {right->i, right->k, right->u};
  double* out = malloc(sizeof(double) * 2 * nn);
  elem_t res = {right->i, right->k, out};
  memcpy(out, right->u, sizeof(double) * 2 * nn);
  apply_b(S, &l, &res, op_index);  /* res <- l (.) res */
  memcpy(dst->u, out, sizeof(double) * 2 * nn);
  dst->id = 0;
  dst->i = res.i;
  dst->k = res.k;
  free(out);
  (void)r;
}

static velem_t* velems(int n, size_t nn) {
  velem_t* v = calloc((size_t)n, sizeof(velem_t));
  for (int e = 0; e < n; ++e) {
    v[e].id = 1;
    v[e].u = calloc(2 * nn, sizeof(double));
  }
  return v;
}

static void velems_free(velem_t* v, int n) {
  for (int e = 0; e < n; ++e) free(v[e].u);
  free(v);
}

/* Blelloch (algorithm "blelloch"), the exclusive scan with the identity element, for any M:
   the M neighbour results padded with identities to a power of two n2. Up-sweep, d = 1, 2, ...,
   n2/2: a[j] <- a[j-d] (.) a[j] for j = 2d-1, 4d-1, ... Down-sweep: the root's total is kept and
   the root becomes the identity; for d = n2/2, ..., 1 and the same j: the left child a[j-d]
   takes the parent's value a[j], and a[j] becomes the parent's value combined with the left
   child's old value (parent (.) left: the order of a non-commutative operator; the listing
   writes them the other way round). Then a[m] = x_0 (.) ... (.) x_{m-1}, so y_m = a[m+1] for
   m < M-1 and y_{M-1} is the kept total. Registrations are numbered level by level, j
   increasing; combinations with the identity are not registrations. Returns their count. */
static int scan_blelloch(series_ctx* S, elem_t* x, int M) {
  size_t nn = (size_t)S->nf * S->nf;
  int n2 = 1;
  while (n2 < M) n2 *= 2;
  velem_t* a = velems(n2, nn);
  for (int m = 0; m < M; ++m) {
    a[m].id = 0;
    a[m].i = x[m].i;
    a[m].k = x[m].k;
    memcpy(a[m].u, x[m].u, sizeof(double) * 2 * nn);
  }
  int ops = 0;
  int* reg = malloc(sizeof(int) * (size_t)n2);
  for (int d = 1; d < n2; d *= 2) {
    int cnt = 0;
    for (int j = 2 * d - 1; j < n2; j += 2 * d) reg[j] = (!a[j - d].id && !a[j].id) ? ops + cnt++ : -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 2 * d - 1; j < n2; j += 2 * d) combine(S, &a[j - d], &a[j], &a[j], reg[j]);
    ops += cnt;
  }
  velem_t total = a[n2 - 1];
  total.u = malloc(sizeof(double) * 2 * nn);
  memcpy(total.u, a[n2 - 1].u, sizeof(double) * 2 * nn);
  a[n2 - 1].id = 1;
  velem_t* t = velems(n2, nn);
  for (int d = n2 / 2; d >= 1; d /= 2) {
    int cnt = 0;
    for (int j = 2 * d - 1; j < n2; j += 2 * d) {
      /* t = left child, left child <- parent (copies; the combine then reads t) */
      t[j].id = a[j - d].id;
      t[j].i = a[j - d].i;
      t[j].k = a[j - d].k;
      memcpy(t[j].u, a[j - d].u, sizeof(double) * 2 * nn);
      a[j - d].id = a[j].id;
      a[j - d].i = a[j].i;
      a[j - d].k = a[j].k;
      memcpy(a[j - d].u, a[j].u, sizeof(double) * 2 * nn);
      reg[j] = (!a[j].id && !t[j].id) ? ops + cnt++ : -1;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 2 * d - 1; j < n2; j += 2 * d) combine(S, &a[j], &t[j], &a[j], reg[j]);
    ops += cnt;
  }
  for (int m = 0; m < M; ++m) {  /* inclusive values into the elements */
    const velem_t* src = m + 1 < M ? &a[m + 1] : &total;
    x[m].i = src->i;
    x[m].k = src->k;
    memcpy(x[m].u, src->u, sizeof(double) * 2 * nn);
  }
  free(total.u);
  free(reg);
  velems_free(t, n2);
  velems_free(a, n2);
  return ops;
}

/* Alternative strategy of the distributed chapter (algorithm "distributed_alternative_parallel")
   on P workers (0: ceil(sqrt(M))) with the chunks of the general strategy. Reduce: each worker
   folds its chunk into a total T_I = x_l (.) ... (.) x_r, the elements untouched. Global stage:
   the totals scanned with Brent-Kung in place, so T_{I-1} is everything before chunk I. Rescan:
   each worker runs the serial scan of its chunk from that value, y_l = T_{I-1} (.) x_l (worker
   0: y_l = x_l), y_j = y_{j-1} (.) x_j. Registrations are numbered stage by stage, each stage's
   steps in order and the workers of a step in order. Returns their count. */
static int scan_reduce_then_scan(series_ctx* S, elem_t* x, int M, int workers) {
  size_t nn = (size_t)S->nf * S->nf;
  int P = workers > 0 ? workers : (int)ceil(sqrt((double)M));
  if (P > M) P = M;
  int* l = malloc(sizeof(int) * P);
  int* r = malloc(sizeof(int) * P);
  int K = M / P, extra = M % P, at = 0, kmax = 0;
  for (int I = 0; I < P; ++I) {
    int k = K + (I < extra ? 1 : 0);
    l[I] = at;
    r[I] = at + k - 1;
    at += k;
    if (k > kmax) kmax = k;
  }
  velem_t* T = velems(P, nn);
  velem_t* v = velems(M, nn);
  for (int m = 0; m < M; ++m) {
    v[m].id = 0;
    v[m].i = x[m].i;
    v[m].k = x[m].k;
    memcpy(v[m].u, x[m].u, sizeof(double) * 2 * nn);
  }
  for (int I = 0; I < P; ++I) {
    T[I].id = 0;
    T[I].i = v[l[I]].i;
    T[I].k = v[l[I]].k;
    memcpy(T[I].u, v[l[I]].u, sizeof(double) * 2 * nn);
  }
  int ops = 0;
  for (int st = 1; st < kmax; ++st) {  /* reduce */
    int cnt = 0;
    int* idx = malloc(sizeof(int) * P);
    for (int I = 0; I < P; ++I) idx[I] = l[I] + st <= r[I] ? ops + cnt++ : -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int I = 0; I < P; ++I)
      if (idx[I] >= 0) combine(S, &T[I], &v[l[I] + st], &T[I], idx[I]);
    ops += cnt;
    free(idx);
  }
  for (int d = 1; d < P; d *= 2) {  /* global stage: Brent-Kung over the totals */
    int cnt = 0;
    for (int j = 2 * d - 1; j < P; j += 2 * d) ++cnt;
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < cnt; ++q) {
      int j = 2 * d - 1 + q * 2 * d;
      combine(S, &T[j - d], &T[j], &T[j], ops + q);
    }
    ops += cnt;
  }
  int dtop = 1;
  while (dtop * 2 < P) dtop *= 2;
  for (int d = dtop; d >= 1; d /= 2) {
    int cnt = 0;
    for (int j = 3 * d - 1; j < P; j += 2 * d) ++cnt;
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < cnt; ++q) {
      int j = 3 * d - 1 + q * 2 * d;
      combine(S, &T[j - d], &T[j], &T[j], ops + q);
    }
    ops += cnt;
  }
  for (int st = 0; st < kmax; ++st) {  /* rescan, the chunks side by side */
    int cnt = 0;
    int* idx = malloc(sizeof(int) * P);
    for (int I = 0; I < P; ++I)
      idx[I] = (l[I] + st <= r[I] && !(st == 0 && I == 0)) ? ops + cnt++ : -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int I = 0; I < P; ++I) {
      if (idx[I] < 0) continue;
      int j = l[I] + st;
      const velem_t* left = st == 0 ? &T[I - 1] : &v[j - 1];
      combine(S, left, &v[j], &v[j], idx[I]);
    }
    ops += cnt;
    free(idx);
  }
  for (int m = 0; m < M; ++m) {
    x[m].i = v[m].i;
    x[m].k = v[m].k;
    memcpy(x[m].u, v[m].u, sizeof(double) * 2 * nn);
  }
  velems_free(v, M);
  velems_free(T, P);
  free(l);
  free(r);
  return ops;
}

/* force_a ([N-1][OR_MAX_LEVELS]) and force_b ([ops][OR_MAX_LEVELS]), rungs_a ([N-1][rung_cap])
   and rungs_b ([ops][rung_cap]), each may be NULL: the replayed decisions of or_register_f for
   every neighbour registration and B application. */
int or_series_f(const double* frames, int N, int nf, const or_params* p, int scan, int workers,
                const int* force_a, const int* force_b, const unsigned char* rungs_a,
                const unsigned char* rungs_b, int rung_cap, double* u_out, or_stats* a_stats,
                or_stats* b_stats, int* b_pairs, int threads) {
  if (N < 1) return -1;
  size_t nn = (size_t)nf * nf;
  memset(u_out, 0, sizeof(double) * 2 * nn);
  int M = N - 1;
  if (M == 0) return 0;
  elem_t* x = malloc(sizeof(elem_t) * M);
  int err = 0;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
  for (int m = 0; m < M; ++m) {
    x[m].i = m;
    x[m].k = m + 1;
    x[m].u = u_out + (size_t)(m + 1) * 2 * nn;
  }
  /* Preprocessing: neighbour registrations are independent. */
#pragma omp parallel for schedule(dynamic, 1)
  for (int m = 0; m < M; ++m) {
    or_stats st;
    int rc = or_register_f(frames + (size_t)m * nn, frames + (size_t)(m + 1) * nn, nf, NULL, p,
                           force_a ? force_a + (size_t)m * OR_MAX_LEVELS : NULL,
                           rungs_a ? rungs_a + (size_t)m * rung_cap : NULL, rung_cap, x[m].u,
                           &st, NULL, 0, NULL);
    if (rc != 0) err = rc;
    if (a_stats) a_stats[m] = st;
  }
  if (err) {
    free(x);
    return err;
  }
  series_ctx S = {frames, nf, p, b_stats, b_pairs, force_b, rungs_b, rung_cap, 0, 0};
  int ops = 0;
  if (scan == OR_SCAN_SEQUENTIAL) {
    /* y_0 = x_0, y_m = y_{m-1} (.) x_m */
    for (int m = 1; m < M; ++m) apply_b(&S, &x[m - 1], &x[m], ops++);
  } else if (scan == OR_SCAN_BRENT_KUNG) {
    /* Up-sweep: x_j <- x_{j-d} (.) x_j for j = 2d-1, 4d-1, ... */
    for (int d = 1; d < M; d *= 2) {
      int cnt = 0;
      for (int j = 2 * d - 1; j < M; j += 2 * d) ++cnt;
#pragma omp parallel for schedule(dynamic, 1)
      for (int q = 0; q < cnt; ++q) {
        int j = 2 * d - 1 + q * 2 * d;
        apply_b(&S, &x[j - d], &x[j], ops + q);
      }
      ops += cnt;
    }
    /* Down-sweep: x_j <- x_{j-d} (.) x_j for j = 3d-1, 5d-1, ..., d halving to 1. */
    int dtop = 1;
    while (dtop * 2 < M) dtop *= 2;
    for (int d = dtop; d >= 1; d /= 2) {
      int cnt = 0;
      for (int j = 3 * d - 1; j < M; j += 2 * d) ++cnt;
#pragma omp parallel for schedule(dynamic, 1)
      for (int q = 0; q < cnt; ++q) {
        int j = 3 * d - 1 + q * 2 * d;
        apply_b(&S, &x[j - d], &x[j], ops + q);
      }
      ops += cnt;
    }
  } else if (scan == OR_SCAN_KOGGE_STONE) {
    /* Step d = 1, 2, 4, ...: x_j <- x_{j-d} (.) x_j for every j >= d, each with the values of
       the previous step (the double buffering the Kogge-Stone section describes); the listing's
       lower bound of j is read as d. Taking j from the right end down reads every x_{j-d}
       before this step rewrites it, which is that double buffering without a second array. */
    for (int d = 1; d < M; d *= 2)
      for (int j = M - 1; j >= d; --j) apply_b(&S, &x[j - d], &x[j], ops++);
  } else if (scan == OR_SCAN_SKLANSKY) {
    /* Step d = 1, 2, 4, ...: in every block of 2d elements, each of the upper d elements takes
       the last element of the lower d as its left operand (Sklansky listing: sources j =
       d-1, 3d-1, ..., destinations j+1 .. j+d). No op of a step rewrites a source. */
    for (int d = 1; d < M; d *= 2) {
      int cnt = 0;
      for (int j = d - 1; j < M; j += 2 * d)
        for (int k = 0; k < d && j + k + 1 < M; ++k) ++cnt;
      int* src = malloc(sizeof(int) * (cnt > 0 ? cnt : 1));
      int* dst = malloc(sizeof(int) * (cnt > 0 ? cnt : 1));
      int q = 0;
      for (int j = d - 1; j < M; j += 2 * d)
        for (int k = 0; k < d && j + k + 1 < M; ++k) {
          src[q] = j;
          dst[q] = j + k + 1;
          ++q;
        }
#pragma omp parallel for schedule(dynamic, 1)
      for (int t = 0; t < cnt; ++t) apply_b(&S, &x[src[t]], &x[dst[t]], ops + t);
      ops += cnt;
      free(src);
      free(dst);
    }
  } else if (scan == OR_SCAN_GENERAL) {
    ops = scan_general(&S, x, M, workers);
  } else if (scan == OR_SCAN_BLELLOCH) {
    ops = scan_blelloch(&S, x, M);
  } else if (scan == OR_SCAN_REDUCE_THEN_SCAN) {
    ops = scan_reduce_then_scan(&S, x, M, workers);
  } else {
    free(x);
    return -1;
  }
  for (int m = 0; m < M; ++m)
    if (x[m].i != 0 || x[m].k != m + 1) S.err = -4;
  free(x);
  return S.err ? S.err : ops;
}

int or_series(const double* frames, int N, int nf, const or_params* p, int scan, int workers,
              double* u_out, or_stats* a_stats, or_stats* b_stats, int* b_pairs,
              int threads) {
  return or_series_f(frames, N, nf, p, scan, workers, NULL, NULL, NULL, NULL, 0, u_out,
                     a_stats, b_stats, b_pairs, threads);
}

int or_register_rigid(const double* R, const double* T, int nf, const double* p_init,
                      const or_params* pr, double* p_out, or_stats* st) {
  return or_register_rigid_f(R, T, nf, p_init, pr, NULL, NULL, 0, p_out, st);
}
