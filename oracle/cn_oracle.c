/*
 * CPU oracle for the Crank-Nicolson tridiagonal path (TEST INFRASTRUCTURE ONLY).
 *
 * This file is the plain, slow, obviously correct reference that the GPU path is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product library never links or calls it.  It shares no
 * code, header, table or helper with the HIP path.
 *
 * Arithmetic: IEEE FP64, C99 double complex (the compiler's own complex division),
 * built with -O2 -ffp-contract=off and no fast-math.
 *
 * Paper: Lutsyshyn, Navarrete, Bauer, "The N-shaped partition method: A novel parallel
 * implementation of the Crank Nicolson algorithm" (arXiv 2205.00856).
 *   - Sec. 2, Eqs. (2)-(4): CN step  T psi(t+dt) = T^dagger psi(t),  T = 1 + i dt H / 2.
 *   - Sec. 4, Eq. (5): row i reads  b_i psi_{i-1} + a_i psi_i + c_i psi_{i+1} = d_i,
 *     b_1 = c_n = 0 (rows are 0-based here: b[0] and c[n-1] are never read).
 *   - Sec. 2 (last paragraph) and the RS stage of Table 1: the Thomas elimination
 *       r_i = -b_i / a_{i-1};  a_i += r_i c_{i-1};  d_i += r_i d_{i-1}
 *       psi_n = d_n / a_n;     psi_i = (d_i - c_i psi_{i+1}) / a_i
 *     with no pivoting.  The N-shaped method reaches exactly this x = T^{-1} d up to
 *     rounding (Appendix I: a reordering of the same elementary row operations), so the
 *     oracle is the serial elimination written out.
 *
 * Discretisation (fixed by the workloads, not by the paper): three-point Laplacian on a
 * uniform grid with Dirichlet walls psi_{-1} = psi_n = 0,
 *   (H psi)_j = (1/dx^2 + V_j) psi_j - (psi_{j-1} + psi_{j+1}) / (2 dx^2),
 * so with tau = dt/2 and kappa = tau/(2 dx^2):
 *   T   : diagonal 1 + i tau (1/dx^2 + V_j),  off-diagonals -i kappa,
 *   rhs : d_j = (1 - i tau (1/dx^2 + V_j)) psi_j + i kappa (psi_{j-1} + psi_{j+1}).
 * For real V the explicit operator 1 - i tau H equals T^dagger (Sec. 2).  A length-gauge
 * field adds x_j * E to V_j when xgrid is given.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Thomas elimination (RS stage of Table 1 applied to the whole system).
 * a, b, c, d: length n, read only.  x: length n, output.  w: length 2n workspace.
 * Returns 0 on success, 1 if a pivot is zero or not finite. */
int oracle_thomas(int64_t n, const cplx* a, const cplx* b, const cplx* c, const cplx* d,
                  cplx* x, cplx* w) {
  if (n <= 0) return 0;
  cplx* ap = w;      /* eliminated diagonal */
  cplx* dp = w + n;  /* eliminated right-hand side */
  ap[0] = a[0];
  dp[0] = d[0];
  for (int64_t i = 1; i < n; ++i) {
    if (ap[i - 1] == 0.0 || !isfinite(creal(ap[i - 1])) || !isfinite(cimag(ap[i - 1])))
      return 1;
    cplx r = -b[i] / ap[i - 1];
    ap[i] = a[i] + r * c[i - 1];
    dp[i] = d[i] + r * dp[i - 1];
  }
  if (ap[n - 1] == 0.0) return 1;
  x[n - 1] = dp[n - 1] / ap[n - 1];
  for (int64_t i = n - 2; i >= 0; --i) x[i] = (dp[i] - c[i] * x[i + 1]) / ap[i];
  return 0;
}

/* Many independent systems packed back to back: system s owns rows
 * offsets[s] .. offsets[s+1]-1 of every array.  One system per host thread. */
int oracle_thomas_batched(int64_t batch, const int64_t* offsets, const cplx* a, const cplx* b,
                          const cplx* c, const cplx* d, cplx* x, int nthreads) {
  int bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
#endif
  for (int64_t s = 0; s < batch; ++s) {
    int64_t o = offsets[s], len = offsets[s + 1] - offsets[s];
    cplx* w = (cplx*)malloc(sizeof(cplx) * (size_t)(2 * (len > 0 ? len : 1)));
    bad |= oracle_thomas(len, a + o, b + o, c + o, d + o, x + o, w);
    free(w);
  }
  return bad;
}

/* Coefficients of T = 1 + i tau H (Sec. 2, Eq. (4) with the Laplacian above).
 * xgrid may be NULL (no field term).  W may be NULL; else the potential is v - i W
 * (an absorbing, non-Hermitian H), so that T's diagonal gains + tau W_j. */
void oracle_cn_coeffs_w(int64_t n, const double* V, double dx, double dt, const double* xgrid,
                        double E, const double* W, cplx* a, cplx* b, cplx* c) {
  double tau = 0.5 * dt;
  double kappa = tau / (2.0 * dx * dx);
  for (int64_t j = 0; j < n; ++j) {
    double v = V[j] + (xgrid ? xgrid[j] * E : 0.0);
    cplx h = (1.0 / (dx * dx) + v) - I * (W ? W[j] : 0.0); /* diagonal of H */
    a[j] = 1.0 + I * tau * h;
    b[j] = (j == 0) ? 0.0 : -I * kappa;
    c[j] = (j == n - 1) ? 0.0 : -I * kappa;
  }
}

void oracle_cn_coeffs(int64_t n, const double* V, double dx, double dt, const double* xgrid,
                      double E, cplx* a, cplx* b, cplx* c) {
  oracle_cn_coeffs_w(n, V, dx, dt, xgrid, E, NULL, a, b, c);
}

/* Explicit forward half-step d = (1 - i tau H) psi (Sec. 2, Eq. (3)).  For a Hermitian H this
 * operator is T^dagger; with the absorbing term (W non-NULL) it is 1 - i tau H, not T^dagger:
 * the step stays the Cayley form (1 + i tau H)^{-1} (1 - i tau H) of exp(-i dt H). */
void oracle_cn_rhs_w(int64_t n, const cplx* psi, const double* V, double dx, double dt,
                     const double* xgrid, double E, const double* W, cplx* d) {
  double tau = 0.5 * dt;
  double kappa = tau / (2.0 * dx * dx);
  for (int64_t j = 0; j < n; ++j) {
    double v = V[j] + (xgrid ? xgrid[j] * E : 0.0);
    cplx h = (1.0 / (dx * dx) + v) - I * (W ? W[j] : 0.0);
    cplx left = (j > 0) ? psi[j - 1] : 0.0;
    cplx right = (j < n - 1) ? psi[j + 1] : 0.0;
    d[j] = (1.0 - I * tau * h) * psi[j] + I * kappa * (left + right);
  }
}

void oracle_cn_rhs(int64_t n, const cplx* psi, const double* V, double dx, double dt,
                   const double* xgrid, double E, cplx* d) {
  oracle_cn_rhs_w(n, psi, V, dx, dt, xgrid, E, NULL, d);
}

/* One CN step: d = (1 - i tau H) psi_in, then T psi_out = d (Sec. 2, Eqs. (3)-(4)).
 * psi_out may alias psi_in.  W may be NULL.  Returns the Thomas status. */
int oracle_cn_step_w(int64_t n, const double* V, double dx, double dt, const double* xgrid,
                     double E, const double* W, const cplx* psi_in, cplx* psi_out) {
  cplx* buf = (cplx*)malloc(sizeof(cplx) * (size_t)(6 * n));
  cplx *a = buf, *b = buf + n, *c = buf + 2 * n, *d = buf + 3 * n, *w = buf + 4 * n;
  oracle_cn_coeffs_w(n, V, dx, dt, xgrid, E, W, a, b, c);
  oracle_cn_rhs_w(n, psi_in, V, dx, dt, xgrid, E, W, d);
  int st = oracle_thomas(n, a, b, c, d, psi_out, w);
  free(buf);
  return st;
}

int oracle_cn_step(int64_t n, const double* V, double dx, double dt, const double* xgrid,
                   double E, const cplx* psi_in, cplx* psi_out) {
  return oracle_cn_step_w(n, V, dx, dt, xgrid, E, NULL, psi_in, psi_out);
}

/* nsteps CN steps in place.  E may be NULL (no field); else E[k] is the field of step k,
 * used on both sides of step k (midpoint sample).  W may be NULL. */
int oracle_cn_propagate_w(int64_t n, const double* V, double dx, double dt, int64_t nsteps,
                          const double* xgrid, const double* E, const double* W, cplx* psi) {
  int st = 0;
  for (int64_t k = 0; k < nsteps; ++k)
    st |= oracle_cn_step_w(n, V, dx, dt, xgrid, E ? E[k] : 0.0, W, psi, psi);
  return st;
}

int oracle_cn_propagate(int64_t n, const double* V, double dx, double dt, int64_t nsteps,
                        const double* xgrid, const double* E, cplx* psi) {
  return oracle_cn_propagate_w(n, V, dx, dt, nsteps, xgrid, E, NULL, psi);
}

/* One CN step for each of many packed systems (own dx each), one system per thread. */
int oracle_cn_step_batched(int64_t batch, const int64_t* offsets, const double* V,
                           const double* dx, double dt, const cplx* psi_in, cplx* psi_out,
                           int nthreads) {
  int bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
#endif
  for (int64_t s = 0; s < batch; ++s) {
    int64_t o = offsets[s], len = offsets[s + 1] - offsets[s];
    bad |= oracle_cn_step(len, V + o, dx[s], dt, NULL, 0.0, psi_in + o, psi_out + o);
  }
  return bad;
}

/* One Lie-split ADI step on an ny x nx grid stored row-major (x fastest):
 * every row (fixed y) takes a full 1D CN step along x with potential V/2 and spacing dx,
 * then every column takes one along y with V/2 and spacing dy.  In place. */
int oracle_adi_step(int64_t nx, int64_t ny, const double* V, double dx, double dy, double dt,
                    cplx* psi, int nthreads) {
  int bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(| : bad)
#endif
  for (int64_t y = 0; y < ny; ++y) {
    double* vh = (double*)malloc(sizeof(double) * (size_t)nx);
    for (int64_t x = 0; x < nx; ++x) vh[x] = 0.5 * V[y * nx + x];
    bad |= oracle_cn_step(nx, vh, dx, dt, NULL, 0.0, psi + y * nx, psi + y * nx);
    free(vh);
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : bad)
#endif
  for (int64_t x = 0; x < nx; ++x) {
    double* vh = (double*)malloc(sizeof(double) * (size_t)ny);
    cplx* col = (cplx*)malloc(sizeof(cplx) * (size_t)ny);
    for (int64_t y = 0; y < ny; ++y) {
      vh[y] = 0.5 * V[y * nx + x];
      col[y] = psi[y * nx + x];
    }
    bad |= oracle_cn_step(ny, vh, dy, dt, NULL, 0.0, col, col);
    for (int64_t y = 0; y < ny; ++y) psi[y * nx + x] = col[y];
    free(col);
    free(vh);
  }
  return bad;
}

/* Reverse mode of x = T^{-1} d (plain definition).  With G the gradient of a real loss
 * with respect to x in the (d/dRe + i d/dIm) convention:
 *   lambda = T^{-H} G            (gradient with respect to d)
 *   ga_i = -lambda_i conj(x_i),  gb_i = -lambda_i conj(x_{i-1}),  gc_i = -lambda_i conj(x_{i+1})
 * T^H is tridiagonal with diagonal conj(a_i), sub-diagonal conj(c_{i-1}) and
 * super-diagonal conj(b_{i+1}); it is solved with the same elimination as above.
 * Any of ga, gb, gc may be NULL.  gb[0] and gc[n-1] are set to zero. */
int oracle_thomas_adjoint(int64_t n, const cplx* a, const cplx* b, const cplx* c, const cplx* x,
                          const cplx* G, cplx* lam, cplx* ga, cplx* gb, cplx* gc) {
  cplx* buf = (cplx*)malloc(sizeof(cplx) * (size_t)(5 * n));
  cplx *ah = buf, *bh = buf + n, *ch = buf + 2 * n, *w = buf + 3 * n;
  for (int64_t i = 0; i < n; ++i) {
    ah[i] = conj(a[i]);
    bh[i] = (i > 0) ? conj(c[i - 1]) : 0.0;
    ch[i] = (i < n - 1) ? conj(b[i + 1]) : 0.0;
  }
  int st = oracle_thomas(n, ah, bh, ch, G, lam, w);
  for (int64_t i = 0; i < n; ++i) {
    if (ga) ga[i] = -lam[i] * conj(x[i]);
    if (gb) gb[i] = (i > 0) ? -lam[i] * conj(x[i - 1]) : 0.0;
    if (gc) gc[i] = (i < n - 1) ? -lam[i] * conj(x[i + 1]) : 0.0;
  }
  free(buf);
  return st;
}

/* Reverse mode of nsteps CN steps psi_{k+1} = T_k^{-1} B_k psi_k, T_k = 1 + i tau H_k and
 * B_k = 1 - i tau H_k, with H_k = H_0 + diag(V + xgrid * E[k] - i W) (xgrid/E and W may be
 * NULL).  Plain form: every state is stored (memory n*(nsteps+1)), then the adjoint recursion
 * runs backwards:
 *   lambda_k = T_k^{-H} G_{k+1};   G_k = B_k^H lambda_k
 *   dL/dV_j  += tau * Im(conj(lambda_k,j) (psi_{k,j} + psi_{k+1,j}))
 *   dL/dE_k   = sum_j x_j * tau * Im(conj(lambda_k,j) (psi_{k,j} + psi_{k+1,j}))
 * (V enters T as + i tau dV and B as - i tau dV, so d psi_{k+1} = T_k^{-1} (-i tau dV)
 * (psi_k + psi_{k+1})).  For real potentials B_k^H = T_k; with W, B_k^H has the diagonal
 * 1 + i tau conj(h_j) = 1 - tau W_j + i tau (1/dx^2 + v_j) and the off-diagonals -i kappa.
 * G_T is the loss gradient at the final state (convention as in oracle_thomas_adjoint);
 * on return gpsi0 holds the gradient with respect to psi_0.  dV (length n) and dE (length
 * nsteps, may be NULL) are overwritten. */
int oracle_cn_propagate_grad_w(int64_t n, const double* V, double dx, double dt, int64_t nsteps,
                               const double* xgrid, const double* E, const double* W,
                               const cplx* psi0, const cplx* G_T, cplx* gpsi0, double* dV,
                               double* dE) {
  double tau = 0.5 * dt;
  double kappa = tau / (2.0 * dx * dx);
  cplx* states = (cplx*)malloc(sizeof(cplx) * (size_t)(n * (nsteps + 1)));
  cplx* buf = (cplx*)malloc(sizeof(cplx) * (size_t)(6 * n));
  cplx *a = buf, *b = buf + n, *c = buf + 2 * n, *lam = buf + 3 * n, *g = buf + 4 * n;
  int st = 0;
  memcpy(states, psi0, sizeof(cplx) * (size_t)n);
  for (int64_t k = 0; k < nsteps; ++k)
    st |= oracle_cn_step_w(n, V, dx, dt, xgrid, E ? E[k] : 0.0, W, states + k * n,
                           states + (k + 1) * n);
  memcpy(g, G_T, sizeof(cplx) * (size_t)n);
  for (int64_t j = 0; j < n; ++j) dV[j] = 0.0;
  for (int64_t k = nsteps - 1; k >= 0; --k) {
    double Ek = E ? E[k] : 0.0;
    const cplx* pk = states + k * n;
    const cplx* pk1 = states + (k + 1) * n;
    oracle_cn_coeffs_w(n, V, dx, dt, xgrid, Ek, W, a, b, c);
    st |= oracle_thomas_adjoint(n, a, b, c, pk1, g, lam, NULL, NULL, NULL);
    double acc = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double t = tau * cimag(conj(lam[j]) * (pk[j] + pk1[j]));
      dV[j] += t;
      if (xgrid) acc += xgrid[j] * t;
    }
    if (dE) dE[k] = acc;
    /* G_k = B_k^H lambda_k, B_k = 1 - i tau H_k: diagonal conj(1 - i tau h_j), off-diagonals
     * conj(i kappa) */
    for (int64_t j = 0; j < n; ++j) {
      double v = V[j] + (xgrid ? xgrid[j] * Ek : 0.0);
      cplx h = (1.0 / (dx * dx) + v) - I * (W ? W[j] : 0.0);
      cplx s = conj(1.0 - I * tau * h) * lam[j];
      if (j > 0) s += conj(I * kappa) * lam[j - 1];
      if (j < n - 1) s += conj(I * kappa) * lam[j + 1];
      g[j] = s;
    }
  }
  memcpy(gpsi0, g, sizeof(cplx) * (size_t)n);
  free(buf);
  free(states);
  return st;
}

int oracle_cn_propagate_grad(int64_t n, const double* V, double dx, double dt, int64_t nsteps,
                             const double* xgrid, const double* E, const cplx* psi0,
                             const cplx* G_T, cplx* gpsi0, double* dV, double* dE) {
  return oracle_cn_propagate_grad_w(n, V, dx, dt, nsteps, xgrid, E, NULL, psi0, G_T, gpsi0, dV,
                                    dE);
}

/* Partial-wave (radial) Crank-Nicolson step of the kind Sec. 3 describes for atoms in strong
 * fields expanded in spherical harmonics: radial functions psi_l(r_j), l = l0 .. l0+nl-1, on
 * r_j = j dr (j = 1..nr, psi = 0 at r = 0 and r = (nr+1) dr), stored l-major:
 * psi[(l - l0) * nr + j - 1].  One Lie-split step of dt:
 *  1. for every l, a CN step in r with H_l = -1/2 d^2/dr^2 + V(r) + l(l+1)/(2 r^2);
 *  2. for every r_j, a CN step in l with the length-gauge coupling H_E = E r_j C, where C is
 *     the matrix of cos(theta) between the m = 0 spherical harmonics, tridiagonal in l:
 *     C_{l,l+1} = C_{l+1,l} = (l+1) / sqrt((2l+1)(2l+3)).
 * Both parts are CN steps (1 + i dt/2 H)^{-1} (1 - i dt/2 H) with a Hermitian H. */
static double coupling_c(int64_t l) {
  return (double)(l + 1) / sqrt((double)(2 * l + 1) * (double)(2 * l + 3));
}

int oracle_radial_step(int64_t nr, int64_t l0, int64_t nl, const double* V, double dr,
                       double dt, double E, cplx* psi) {
  int bad = 0;
  double* veff = (double*)malloc(sizeof(double) * (size_t)nr);
  for (int64_t k = 0; k < nl; ++k) {
    const double l = (double)(l0 + k);
    for (int64_t j = 0; j < nr; ++j) {
      const double r = (double)(j + 1) * dr;
      veff[j] = V[j] + l * (l + 1.0) / (2.0 * r * r);
    }
    bad |= oracle_cn_step(nr, veff, dr, dt, NULL, 0.0, psi + k * nr, psi + k * nr);
  }
  free(veff);
  const double tau = 0.5 * dt;
  cplx* buf = (cplx*)malloc(sizeof(cplx) * (size_t)(7 * nl));
  cplx *a = buf, *b = buf + nl, *c = buf + 2 * nl, *d = buf + 3 * nl, *x = buf + 4 * nl,
       *w = buf + 5 * nl;
  for (int64_t j = 0; j < nr; ++j) {
    const double r = (double)(j + 1) * dr;
    for (int64_t k = 0; k < nl; ++k) {
      /* T = 1 + i tau E r C: off-diagonals i tau E r c */
      a[k] = 1.0;
      b[k] = (k > 0) ? I * tau * E * r * coupling_c(l0 + k - 1) : 0.0;
      c[k] = (k < nl - 1) ? I * tau * E * r * coupling_c(l0 + k) : 0.0;
    }
    for (int64_t k = 0; k < nl; ++k) {
      /* d = (1 - i tau E r C) psi */
      cplx s = psi[k * nr + j];
      if (k > 0) s -= b[k] * psi[(k - 1) * nr + j];
      if (k < nl - 1) s -= c[k] * psi[(k + 1) * nr + j];
      d[k] = s;
    }
    bad |= oracle_thomas(nl, a, b, c, d, x, w);
    for (int64_t k = 0; k < nl; ++k) psi[k * nr + j] = x[k];
  }
  free(buf);
  return bad;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
