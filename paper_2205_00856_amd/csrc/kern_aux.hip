// Auxiliary kernels: materialised coefficient assembly and explicit half-step, the gradients
// of a solve, the adjoint accumulation of a Crank-Nicolson step and fixed-order partial sums.
#include "kern_table.hpp"
#include "nshaped_kernels.hpp"

namespace nsd {

// Locate (system, row, element) of flat index t.
__device__ __forceinline__ bool locate(const AuxArgs& A, int64_t t, int64_t& sys, int64_t& r,
                                       int64_t& n, int64_t& e) {
  if (A.offs) {
    if (t >= A.total) return false;
    int64_t lo = 0, hi = A.batch;  // find sys with offs[sys] <= t < offs[sys+1]
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (A.offs[mid] <= t)
        lo = mid;
      else
        hi = mid;
    }
    sys = lo;
    r = t - A.offs[sys];
    n = A.offs[sys + 1] - A.offs[sys];
    e = t;
  } else {
    if (t >= A.n * A.batch) return false;
    sys = t / A.n;
    r = t - sys * A.n;
    n = A.n;
    e = sys * A.bs + r * A.es;
  }
  return true;
}

// a1: coefficients of T = 1 + i tau H
__global__ void k_assemble(AuxArgs A) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, sys, r, n, e;
  if (!locate(A, t, sys, r, n, e)) return;
  const double dx = A.dxs ? A.dxs[sys] : A.dx;
  const double tau = 0.5 * A.dt, idx2 = 1.0 / (dx * dx), kap = tau * 0.5 * idx2;
  const double v = A.vscale * A.V[e] + (A.xg ? A.xg[e] * A.E : 0.0);
  // with the absorbing term -iW in H the diagonal of 1 + i tau H gains + tau W
  A.a[e] = mk(A.W ? fma(tau, A.wscale * A.W[e], 1.0) : 1.0, tau * (idx2 + v));
  A.b[e] = mk(0.0, (r > 0) ? -kap : 0.0);
  A.c[e] = mk(0.0, (r < n - 1) ? -kap : 0.0);
}

// a2: d = (1 - i tau H) psi
__global__ void k_rhs(AuxArgs A) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, sys, r, n, e;
  if (!locate(A, t, sys, r, n, e)) return;
  const int64_t st = A.offs ? 1 : A.es;
  const double dx = A.dxs ? A.dxs[sys] : A.dx;
  const double tau = 0.5 * A.dt, idx2 = 1.0 / (dx * dx), kap = tau * 0.5 * idx2;
  const double w = tau * (idx2 + A.vscale * A.V[e] + (A.xg ? A.xg[e] * A.E : 0.0));
  const cd p = A.psi[e];
  const cd l = csel(r > 0, A.psi[(r > 0) ? e - st : e], czero());
  const cd h = csel(r < n - 1, A.psi[(r < n - 1) ? e + st : e], czero());
  const cd s = cadd(l, h);
  // the diagonal of 1 - i tau H is 1 - tau W - i w (with the absorbing term, not T^dagger's)
  const double f = A.W ? fma(-tau, A.wscale * A.W[e], 1.0) : 1.0;
  const cd q = A.W ? mk(f * p.x, f * p.y) : p;
  A.d[e] = mk(fma(w, p.y, fma(-kap, s.y, q.x)), fma(-w, p.x, fma(kap, s.x, q.y)));
}

// gradients of the solve: ga_i = -lam_i conj(x_i), gb_i = -lam_i conj(x_{i-1}), gc_i = ...
__global__ void k_solve_grads(AuxArgs A) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, sys, r, n, e;
  if (!locate(A, t, sys, r, n, e)) return;
  const int64_t st = A.offs ? 1 : A.es;
  const cd l = A.lam[e];
  if (A.ga) A.ga[e] = cneg(cmul(l, cconj(A.xsol[e])));
  if (A.gb) A.gb[e] = csel(r > 0, cneg(cmul(l, cconj(A.xsol[(r > 0) ? e - st : e]))), czero());
  if (A.gc) A.gc[e] = csel(r < n - 1, cneg(cmul(l, cconj(A.xsol[(r < n - 1) ? e + st : e]))), czero());
}

// adjoint accumulation: q_j = tau Im(conj(lam_j)(psi_n,j + psi_np1,j));
// dV_j += vscale q_j; per-block partial sums of x_j q_j (summed in a fixed order).
__global__ __launch_bounds__(256) void k_adj_accum(AuxArgs A) {
  __shared__ double red[256];
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, sys, r, n, e;
  double part = 0.0;
  if (locate(A, t, sys, r, n, e)) {
    const double tau = 0.5 * A.dt;
    const cd l = A.lam[e];
    const cd s = cadd(A.psi_n[e], A.psi_np1[e]);
    const double q = tau * (l.x * s.y - l.y * s.x);
    if (A.dV) A.dV[e] += A.vscale * q;
    if (A.xg) part = A.xg[e] * q;
  }
  if (!A.dE_part) return;
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) A.dE_part[blockIdx.x] = red[0];
}

// deterministic second stage: workgroup r sets out[r] = sum of the nparts partials in row r of
// part (rows of nparts values), in a fixed order
__global__ __launch_bounds__(256) void k_sum_partials(const double* part, int64_t nparts,
                                                      double* out) {
  __shared__ double red[256];
  part += (int64_t)blockIdx.x * nparts;
  out += blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// RS stage (Table 1) on whole reduced systems, serially: thread s takes reduced system s (rows
// offs[s] .. offs[s+1]-1 of the slot arrays; row k has sub-diagonal DB_{k-1}, diagonal UA_k +
// DA_{k-1}, super-diagonal UC_k and right-hand side UD_k + DD_{k-1}, plus the deferred left
// neighbour term i kap psi_{J-1} of a fused pass when ud_halo is set) and solves it by Thomas's
// elimination: c'_k = c_k / m_k, d'_k = (d_k - b_k d'_{k-1}) / m_k with m_k = a_k - b_k c'_{k-1},
// then x_k = d'_k - c'_k x_{k+1}.  c' and d' go to oU and oD; x to A.x.
__global__ __launch_bounds__(64) void k_rs_serial(KArgs A) {
  const int64_t s = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (s >= A.batch) return;
  const int64_t o0 = A.offs[s], n = A.offs[s + 1] - o0;
  if (n <= 0) return;
  const cd zero = czero();
  double kap = 0.0;
  if (A.ud_halo) kap = cn_kappa(A.dt, A.dxs ? A.dxs[s] : A.dx);
  cd cprev = zero, dprev = zero;
  bool bad = false;
  for (int64_t k = 0; k < n; ++k) {
    const int64_t g = o0 + k;
    cd a = A.sU[3 * g], c = A.sU[3 * g + 1], d = A.sU[3 * g + 2], b = zero;
    if (k > 0) {
      b = A.sD[3 * (g - 1)];
      a = cadd(a, A.sD[3 * (g - 1) + 1]);
      d = cadd(d, A.sD[3 * (g - 1) + 2]);
      if (A.ud_halo) {
        const cd h = A.ud_halo[2 * (g - 1) + 1];
        d = cadd(d, mk(-kap * h.y, kap * h.x));
      }
    }
    if (k == n - 1) c = zero;
    const cd m = csub(a, cmul(b, cprev));
    const cd im = crecip(m);
    cprev = cmul(c, im);
    dprev = cmul(csub(d, cmul(b, dprev)), im);
    A.oU[g] = cprev;
    A.oD[g] = dprev;
  }
  cd x = zero;
  for (int64_t k = n - 1; k >= 0; --k) {
    const int64_t g = o0 + k;
    x = csub(A.oD[g], cmul(A.oU[g], x));
    A.x[g] = x;
    bad |= !cfinite(x);
  }
  if (bad) atomicOr(A.status, 1);
}

// Partial-wave step, radial part: the potential of wave l = l0 + k on r_j = (j + 1) dr,
// V(r_j) + l (l + 1) / (2 r_j^2), for the CN step in r of every wave (l-major, nr per wave).
__global__ void k_radial_veff(AuxArgs A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.n * A.batch) return;
  const int64_t k = t / A.n, j = t - k * A.n;
  const double r = (double)(j + 1) * A.dx;
  const double l = (double)(A.l0 + k);
  A.dV[t] = A.V[j] + l * (l + 1.0) / (2.0 * r * r);
}

// <Y_l0 | cos(theta) | Y_{l+1}0>, the coupling of neighbouring partial waves by a field along z
__device__ __forceinline__ double cos_coupling(int64_t l) {
  return (double)(l + 1) / sqrt((double)(2 * l + 1) * (double)(2 * l + 3));
}

// Partial-wave step, field part: at every r_j the CN step in l with H_E = E r_j C (C the
// tridiagonal coupling of neighbouring waves), materialised: T = 1 + i tau H_E (a = 1,
// b_l = i tau E r c_{l-1}, c_l = i tau E r c_l) and d = (1 - i tau H_E) psi.  Element (wave k,
// point j) at k * nr + j: the systems (one per r_j) are interleaved with stride nr.
__global__ void k_radial_coupling(AuxArgs A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= A.n * A.batch) return;
  const int64_t k = t / A.n, j = t - k * A.n, nl = A.batch;
  const double r = (double)(j + 1) * A.dx;
  const double s = 0.5 * A.dt * A.E * r;  // tau E r
  const double cb = k > 0 ? s * cos_coupling(A.l0 + k - 1) : 0.0;
  const double cc = k < nl - 1 ? s * cos_coupling(A.l0 + k) : 0.0;
  A.a[t] = mk(1.0, 0.0);
  A.b[t] = mk(0.0, cb);
  A.c[t] = mk(0.0, cc);
  // d = psi - b psi_{k-1} - c psi_{k+1} with b, c = i (cb, cc)
  const cd p = A.psi[t];
  const cd lo = k > 0 ? A.psi[t - A.n] : czero();
  const cd hi = k < nl - 1 ? A.psi[t + A.n] : czero();
  A.d[t] = mk(p.x + cb * lo.y + cc * hi.y, p.y - cb * lo.x - cc * hi.x);
}

}  // namespace nsd

namespace nsk {
void reg_aux(Tables& t) {
  t.aux[AUX_ASSEMBLE] = (const void*)&nsd::k_assemble;
  t.aux[AUX_RHS] = (const void*)&nsd::k_rhs;
  t.aux[AUX_SOLVE_GRADS] = (const void*)&nsd::k_solve_grads;
  t.aux[AUX_ADJ_ACCUM] = (const void*)&nsd::k_adj_accum;
  t.aux[AUX_SUM_PARTIALS] = (const void*)&nsd::k_sum_partials;
  t.aux[AUX_RS_SERIAL] = (const void*)&nsd::k_rs_serial;
  t.aux[AUX_RADIAL_VEFF] = (const void*)&nsd::k_radial_veff;
  t.aux[AUX_RADIAL_COUPLING] = (const void*)&nsd::k_radial_coupling;
}
}  // namespace nsk
