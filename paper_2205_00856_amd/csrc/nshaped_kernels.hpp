// Kernels of the N-shaped partition solver (gfx950, FP64 complex).
// Method: arXiv 2205.00856, Sec. 4 (Table 1, nesting Eq. (6)), Sec. 5.3 (fused explicit
// half-step), Sec. 2 (Crank-Nicolson operator).
#pragma once
#include "nshaped_device.hpp"

#include <type_traits>

namespace nsd {

enum Src : int {
  SRC_EXPL = 0,     // explicit a, b, c, d arrays
  SRC_EXPL_CT = 1,  // explicit arrays, conjugate-transposed matrix T^H (adjoint solve)
  SRC_CN = 2,       // Crank-Nicolson operator assembled in-kernel from V, dx, dt (+ x E)
  SRC_SLOTS = 3,    // reduced system of the level below, read from its two slot arrays
  SRC_CNW = 4,      // Crank-Nicolson operator with an absorbing potential, v - i W (H not
                    // Hermitian): T's diagonal 1 + tau W + i tau (...), explicit side 1 - tau W
                    // - i tau (...), off-diagonals -i kappa and +i kappa as in SRC_CN
  SRC_LCOUP = 5     // partial waves: the CN step in l at radial point r = (system + 1) dx with
                    // the field coupling E r C (C_{l,l+1} = (l+1)/sqrt((2l+1)(2l+3)), l = l0 +
                    // row): T = 1 + i tau E r C, explicit side 1 - i tau E r C, both from psi
};
// sources whose rows are the Crank-Nicolson operator assembled in-kernel
__host__ __device__ constexpr bool cn_src(int S) { return S == SRC_CN || S == SRC_CNW; }
// sources whose right-hand side is built from the state's neighbouring rows: a multi-tile pass
// that writes the state in place keeps each tile's first and last row for its neighbours
__host__ __device__ constexpr bool halo_src(int S) { return cn_src(S) || S == SRC_LCOUP; }
enum Phase : int {
  PH_SINGLE = 0,  // the tile holds the whole system: reduce, RS, SS in one pass
  PH_REDUCE = 1,  // first pass of a multi-tile system: reduce, write the tile's slots
  PH_SUBST = 2,   // second pass: re-reduce, take the tile's joint lines from above, SS
  PH_FUSE = 3,    // Crank-Nicolson sequences: PH_SUBST of step n, then PH_REDUCE of step n+1 on
                  // the new state (the tile's joint row defers its left neighbour, see ud_halo)
  PH_RES = 4      // a step of the resident propagation (k_resident): PH_REDUCE's hand-over,
                  // then, once the reduced system is solved in the same launch, PH_SUBST's
                  // substitution (not a phase of the kernel tables)
};

struct KArgs {
  // batch geometry
  int64_t n;              // uniform batch: rows per system
  int64_t ntiles;         // uniform batch: tiles per system
  int64_t es, bs;         // uniform batch: element / batch strides (elements)
  const int64_t* offs;    // uneven batch: CSR row offsets per system (device) or null
  const int64_t* tbase;   // uneven multi-tile: first global tile per system (device) or null
  const int* wg_sys;      // launch list: system of each workgroup (device) or null
  const int* wg_tile;     // launch list: tile of each workgroup
  // explicit sources
  const cd *a, *b, *c, *d;
  // Crank-Nicolson source
  const cd* psi;          // state for the explicit half-step
  const cd* rhs;          // given right-hand side instead of the half-step (or null)
  const double* V;
  const double* xg;
  double vscale, E_mat, E_rhs, dx, dt;
  const double* dxs;
  double E_next;          // PH_FUSE: field of step n+1 (matrix and explicit half-step)
  // reduced-system source (level >= 2)
  const cd* sU;           // 3 values per tile: UA, UC, UD
  const cd* sD;           // 3 values per tile: DB, DA, DD
  // reduced system of a PH_FUSE pass: its tiles reduced the explicit half-step of their joint
  // row without the left neighbour psi_{J-1} (the last row of the tile before, written by
  // another workgroup of the same pass); its contribution i kap psi_{J-1} (kap from dt and
  // dx / dxs) joins the right-hand side here, psi_{J-1} read from the pass's edge rows
  const cd* ud_halo;
  // outputs and hand-over between passes
  cd* x;
  cd* oU;
  cd* oD;
  const cd* psi_if;       // solution of the reduced system (one value per tile)
  cd* halo_out;           // first and last state row of each tile (pass 1)
  const cd* halo_in;
  int* status;
  int xcd_remap;          // uniform single-tile launches: XCD-contiguous system order
  int* queue;             // persistent launch: [next item, workgroups done]
  int nitems;             // persistent launch: number of systems in wg_sys
  // adjoint accumulation fused into the store of lambda (CN source, uniform batches):
  //   q_j = acc_tau Im(conj(lambda_j) (acc_pa_j + acc_pb_j)); acc_dV_j += vscale q_j;
  //   acc_part[tile] = sum over the tile of xg_j q_j (fixed order)
  const cd* acc_pa;
  const cd* acc_pb;
  double* acc_dV;
  double* acc_part;
  double acc_tau;
  int acc_half;           // lambda = (x + the value x overwrites) / 2 instead of x (reverse
                          // recursion on g, where lambda_k = (g_k + g_{k+1}) / 2)
  int64_t batch;          // uniform batch size (column kernel, several right-hand sides)
  int nrhs;               // k_tile_mrhs: right-hand sides per workgroup
  int cshared;            // uniform batch: every system reads the coefficients (a, b, c or V,
                          // xgrid) of system 0 (several right-hand sides of one matrix)
  int rev;                // workgroups take their tiles in reverse launch order, by rounds of 8
                          // (second pass: the tiles the first pass read last are still cached)
  // SRC_CNW: absorbing potential W (layout of V) and its factor; the potential is
  // v - i wscale W (wscale = -1 with dt -> -dt gives the conjugate-transposed operators)
  const double* Wabs;
  double wscale;
  int64_t l0;  // SRC_LCOUP: partial wave of row 0
  // PH_FUSE of one system: the reduced system of the tile joints is solved by the pass's last
  // workgroup (count of workgroups done, zero between launches), or null (a launch of its own)
  int* inl_sync;
};

struct Geo {
  int64_t sys, tile, n, base, es, gt, ntile;
  int64_t cbase;  // first element of the system's coefficients (0 when they are shared)
};

// Launch position of a second-pass workgroup of a one-dimensional grid: the launch order
// reversed in rounds of 8.  Workgroups go to the 8 XCDs round-robin by linear id, so each tile
// keeps the XCD (and the L2) of its first pass while the tiles that pass read last come first.
__device__ __forceinline__ unsigned rev_linear(unsigned L, unsigned G) {
  const unsigned Q = G >> 3;
  if (L >= 8 * Q) return L;
  return 8 * (Q - 1 - (L >> 3)) + (L & 7);
}

template <int PH>
__device__ __forceinline__ Geo geometry(const KArgs& A) {
  Geo g;
  unsigned bx = blockIdx.x;
  const unsigned by = blockIdx.y;
  // second passes only (PH_SUBST, PH_FUSE); the host sets rev for one-dimensional grids
  if constexpr (PH >= 2) {
    if (A.rev) bx = rev_linear(bx, gridDim.x);
  }
  if (A.wg_sys) {
    g.sys = A.wg_sys[bx];
    g.tile = A.wg_tile[bx];
  } else if (A.xcd_remap && gridDim.x == 1) {
    // Workgroups are handed to the 8 XCDs round-robin by linear id; give each XCD a contiguous
    // range of systems so that neighbouring (interleaved) systems share its L2.
    const int64_t B = gridDim.y, id = blockIdx.y, x = id & 7, q = B >> 3, r = B & 7;
    g.sys = x * q + (x < r ? x : r) + (id >> 3);
    g.tile = 0;
  } else {
    g.sys = by;
    g.tile = bx;
  }
  if (A.offs) {
    g.base = A.offs[g.sys];
    g.n = A.offs[g.sys + 1] - g.base;
    g.es = 1;
    if (A.tbase) {
      g.gt = A.tbase[g.sys] + g.tile;
      g.ntile = A.tbase[g.sys + 1] - A.tbase[g.sys];
    } else {
      g.gt = g.sys;
      g.ntile = 1;
    }
  } else {
    g.base = g.sys * A.bs;
    g.n = A.n;
    g.es = A.es;
    g.gt = g.sys * A.ntiles + g.tile;
    g.ntile = A.ntiles;
  }
  g.cbase = A.cshared ? 0 : g.base;
  return g;
}

__device__ __forceinline__ double sel(bool p, double a, double b) { return p ? a : b; }
__device__ __forceinline__ cd sel(bool p, cd a, cd b) { return csel(p, a, b); }

// Interior wavefronts: every row a wavefront touches, its two halo rows included, lies strictly
// inside the system (w0 >= 1 and w0 + 64 M <= n - 1).  Their rows need no clamping and no edge
// selects; IN = true compiles that path, IN = false the general one.
template <bool IN>
__device__ __forceinline__ bool row_in(int64_t r, int64_t n) {
  return IN || r < n;
}
template <bool IN>
__device__ __forceinline__ bool row_pos(int64_t r) {
  return IN || r > 0;
}
template <bool IN>
__device__ __forceinline__ bool row_notlast(int64_t r, int64_t n) {
  return IN || r < n - 1;
}

// Fetch rows w0 + 64k + lane (k < M) and the two halo rows w0-1 (lane 0) and w0+64M (lane 1)
// of a strided array into registers.  Loads are unconditional at a clamped row (n >= 1) and the
// fill value is selected afterwards, so no lane takes a different path.
template <int M, bool IN, typename T>
__device__ __forceinline__ void stage_fetch(const T* g, int64_t es, int64_t w0, int64_t n,
                                            int lane, T fill, T (&v)[M], T& h) {
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const int64_t r = w0 + 64 * k + lane;
    if constexpr (IN) {
      v[k] = sel(true, g[r * es], fill);  // a fresh value (a plain copy defeats promotion)
    } else {
      const T t = g[(r < n ? r : n - 1) * es];
      v[k] = sel(r < n, t, fill);
    }
  }
  const int64_t rr = (lane == 0) ? w0 - 1 : w0 + 64 * M;
  if constexpr (IN) {
    h = sel(true, g[rr * es], fill);
  } else {
    const int64_t rc = rr < 0 ? 0 : (rr < n ? rr : n - 1);
    const T t = g[rc * es];
    h = sel(rr >= 0 && rr < n, t, fill);
  }
}

template <int M, typename T>
__device__ __forceinline__ void stage_put(T* buf, int lane, const T (&v)[M], T h) {
  using S = Stage<M>;
#pragma unroll
  for (int k = 0; k < M; ++k) buf[S::addr(1 + 64 * k + lane)] = v[k];
  if (lane == 0) buf[S::addr(0)] = h;
  if (lane == 1) buf[S::addr(S::QN - 1)] = h;
}

// Read rows J-1 .. J+M of this lane (J = w0 + lane*M) from the staged buffer.
template <int M, typename T>
__device__ __forceinline__ void stage_read(const T* buf, int lane, T (&v)[M + 2]) {
  using S = Stage<M>;
#pragma unroll
  for (int j = 0; j < M + 2; ++j) v[j] = buf[S::addr(lane * M + j)];
}

// registers (coalesced order) -> LDS -> registers (lane-block order)
template <int M, typename T>
__device__ __forceinline__ void transpose_in(T* buf, int lane, const T (&v)[M], T h,
                                             T (&out)[M + 2]) {
  stage_put<M>(buf, lane, v, h);
  wave_sync();
  stage_read<M>(buf, lane, out);
  wave_sync();
}

// ------------------------------------------------------------------ Crank-Nicolson rows
// Raw coalesced loads of one wavefront's rows (state or given right-hand side, V, xgrid).
template <int M, bool XG, bool WA = false>
struct CnRaw {
  cd p[M];
  cd hp;
  double v[M];
  double hv;
  double x[XG ? M : 1];
  double hx;
  double w[WA ? M : 1];  // absorbing potential (SRC_CNW)
  double hw;
};

template <int M, bool XG, bool IN, bool WA>
__device__ __forceinline__ void cn_fetch(const KArgs& A, const Geo& G, int64_t w0, int lane,
                                         CnRaw<M, XG, WA>& r) {
  const cd* src = (A.rhs ? A.rhs : A.psi) + G.base;
  stage_fetch<M, IN>(src, G.es, w0, G.n, lane, czero(), r.p, r.hp);
  stage_fetch<M, IN>(A.V + G.cbase, G.es, w0, G.n, lane, 0.0, r.v, r.hv);
  if constexpr (XG) {
    if (A.xg) stage_fetch<M, IN>(A.xg + G.cbase, G.es, w0, G.n, lane, 0.0, r.x, r.hx);
  }
  if constexpr (WA) stage_fetch<M, IN>(A.Wabs + G.cbase, G.es, w0, G.n, lane, 0.0, r.w, r.hw);
}

// Magnitude of the off-diagonals of T = 1 + i tau H: tau / (2 dx^2) with tau = dt / 2.
__device__ __forceinline__ double cn_kappa(double dt, double dx) {
  return (0.5 * dt) * 0.5 * (1.0 / (dx * dx));
}

// Rows of T = 1 + i tau H and the explicit half-step d = (1 - i tau H) psi (Sec. 2, Eq. (3)),
// fused into the reduction (Sec. 5.3).  The off-diagonals are -i kappa (pure imaginary).
// vp holds psi at rows J-1 .. J+M of this lane (zero outside the system), vv and xv hold V and
// xgrid at the same rows (only J .. J+M-1 are read).
// With WA (SRC_CNW) wv holds the absorbing potential at the same rows: T's diagonal gains
// + tau W and the explicit side's - tau W.
template <int M, bool IN, bool WA = false>
__device__ __forceinline__ void cn_rows(const KArgs& A, const Geo& G, double dx, int64_t J,
                                        const cd (&vp)[M + 2], const double (&vv)[M + 2],
                                        const double (&xv)[M + 2], double Em, double Er,
                                        bool given, cd (&Ar)[M], cd (&Br)[M], cd (&Cr)[M],
                                        cd (&Dr)[M], cd& bK, const double* wv = nullptr) {
  const int64_t n = G.n;
  const double tau = 0.5 * A.dt;
  const double idx2 = 1.0 / (dx * dx);
  const double kap = cn_kappa(A.dt, dx);
  const cd zero = czero();
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int64_t r = J + j;
    const bool ok = row_in<IN>(r, n);
    const double vm = fma(xv[j + 1], Em, A.vscale * vv[j + 1]);
    double tw = 0.0;  // tau W (SRC_CNW)
    if constexpr (WA) tw = ok ? tau * (A.wscale * wv[j + 1]) : 0.0;
    Ar[j] = mk(WA ? 1.0 + tw : 1.0, ok ? tau * (idx2 + vm) : 0.0);
    Br[j] = mk(0.0, (ok && row_pos<IN>(r)) ? -kap : 0.0);
    Cr[j] = mk(0.0, (ok && row_notlast<IN>(r, n)) ? -kap : 0.0);
    if (given) {
      Dr[j] = vp[j + 1];
    } else {
      const double w = tau * (idx2 + fma(xv[j + 1], Er, A.vscale * vv[j + 1]));
      const cd p = vp[j + 1];
      const cd s = cadd(vp[j], vp[j + 2]);
      if constexpr (WA) {
        Dr[j] = csel(ok, mk(fma(-tw, p.x, fma(w, p.y, fma(-kap, s.y, p.x))),
                            fma(-tw, p.y, fma(-w, p.x, fma(kap, s.x, p.y)))), zero);
      } else {
        Dr[j] = csel(ok, mk(fma(w, p.y, fma(-kap, s.y, p.x)), fma(-w, p.x, fma(kap, s.x, p.y))), zero);
      }
    }
  }
  bK = mk(0.0, row_in<IN>(J + M, n) ? -kap : 0.0);
}

template <int M, int W, int PH, bool XG, bool IN, bool WA = false>
__device__ __forceinline__ void cn_build(const KArgs& A, const Geo& G, cd* buf, int64_t w0,
                                         int64_t J, int lane, int wave, CnRaw<M, XG, WA>& raw,
                                         cd (&Ar)[M], cd (&Br)[M], cd (&Cr)[M], cd (&Dr)[M],
                                         cd& bK, cd& first_state, cd& last_state,
                                         double* ayn, double* vkeep = nullptr) {
  if constexpr (PH == PH_SUBST) {
    // the neighbours' edge rows may already hold the new state: take the saved copies
    if (A.rhs == nullptr) {
      if (wave == 0 && lane == 0 && G.tile > 0) raw.hp = A.halo_in[2 * (G.gt - 1) + 1];
      if (wave == W - 1 && lane == 1 && G.tile + 1 < G.ntile) raw.hp = A.halo_in[2 * (G.gt + 1)];
    }
  }
  cd vp[M + 2];
  transpose_in<M>(buf, lane, raw.p, raw.hp, vp);
  double vv[M + 2], xv[M + 2];
  double* bufd = reinterpret_cast<double*>(buf);
  transpose_in<M>(bufd, lane, raw.v, raw.hv, vv);
  bool hasx = false;
  if constexpr (XG) {
    if (A.xg) {
      hasx = true;
      transpose_in<M>(bufd, lane, raw.x, raw.hx, xv);
    }
  }
  if (!hasx) {
#pragma unroll
    for (int j = 0; j < M + 2; ++j) xv[j] = 0.0;
  }
  double wv[WA ? M + 2 : 1];
  if constexpr (WA) transpose_in<M>(bufd, lane, raw.w, raw.hw, wv);
  const double dx = A.dxs ? A.dxs[G.sys] : A.dx;
  cn_rows<M, IN, WA>(A, G, dx, J, vp, vv, xv, A.E_mat, A.E_rhs, A.rhs != nullptr, Ar, Br, Cr,
                     Dr, bK, WA ? wv : nullptr);
  first_state = vp[1];
  last_state = vp[M];
  if (ayn) {
    // PH_FUSE: the diagonal of the next step (field E_next), the same expression as cn_rows
    const double tau = 0.5 * A.dt;
    const double idx2 = 1.0 / (dx * dx);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const double t = tau * (idx2 + fma(xv[j + 1], A.E_next, A.vscale * vv[j + 1]));
      ayn[j] = row_in<IN>(J + j, G.n) ? t : 0.0;
    }
    // (SRC_CNW: the real parts, 1 + tau W, do not change from step to step: the next step takes
    // those of this one)
  }
  if (vkeep) {
    // the resident propagation: the diagonal's imaginary part at any field E is
    // tau (1/dx^2 + vscale v) + (tau x) E; the two terms per row
    const double tau = 0.5 * A.dt;
    const double idx2 = 1.0 / (dx * dx);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const bool ok = row_in<IN>(J + j, G.n);
      vkeep[j] = ok ? tau * (idx2 + A.vscale * vv[j + 1]) : 0.0;
      vkeep[M + j] = ok ? tau * xv[j + 1] : 0.0;
    }
  }
}

// ------------------------------------------------------------------ row assembly per source
// A load at the level of the memory system shared by all XCDs (a relaxed atomic at device
// scope), for values another workgroup of the same launch stored there (st_coh).
__device__ __forceinline__ cd ld_coh(const cd* p) {
  return mk(__hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
            __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// CL (SRC_SLOTS): the slots, edge rows and joint values are read with ld_coh (the resident
// propagation reads them in the launch that stores them).
template <int M, int W, int SRC, int PH, bool IN, bool CL = false>
__device__ __forceinline__ void load_rows(const KArgs& A, const Geo& G, cd* buf, int64_t w0,
                                          int64_t J, int lane, int wave, cd (&Ar)[M],
                                          cd (&Br)[M], cd (&Cr)[M], cd (&Dr)[M], cd& bK,
                                          cd& first_state, cd& last_state,
                                          double* ayn = nullptr) {
  const int64_t n = G.n;
  if constexpr (SRC == SRC_EXPL || SRC == SRC_EXPL_CT) {
    const cd one = mk(1.0, 0.0), zero = czero();
    cd ra[M], rb[M], rc[M], rd[M], ha, hb, hc, hd;
    stage_fetch<M, IN>(A.a + G.cbase, G.es, w0, n, lane, one, ra, ha);
    stage_fetch<M, IN>(A.b + G.cbase, G.es, w0, n, lane, zero, rb, hb);
    stage_fetch<M, IN>(A.c + G.cbase, G.es, w0, n, lane, zero, rc, hc);
    stage_fetch<M, IN>(A.d + G.base, G.es, w0, n, lane, zero, rd, hd);
    cd va[M + 2], vb[M + 2], vc[M + 2], vd[M + 2];
    transpose_in<M>(buf, lane, ra, ha, va);
    transpose_in<M>(buf, lane, rb, hb, vb);
    transpose_in<M>(buf, lane, rc, hc, vc);
    transpose_in<M>(buf, lane, rd, hd, vd);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t r = J + j;
      const bool ok = row_in<IN>(r, n);
      const bool pos = ok && row_pos<IN>(r), notlast = ok && row_notlast<IN>(r, n);
      // (with IN the selects fold to their first operand)
      if constexpr (SRC == SRC_EXPL) {
        Ar[j] = csel(ok, va[j + 1], one);
        Br[j] = csel(pos, vb[j + 1], zero);
        Cr[j] = csel(notlast, vc[j + 1], zero);
      } else {
        // row i of T^H: diagonal conj(a_i), sub conj(c_{i-1}), super conj(b_{i+1})
        Ar[j] = csel(ok, cconj(va[j + 1]), one);
        Br[j] = csel(pos, cconj(vc[j]), zero);
        Cr[j] = csel(notlast, cconj(vb[j + 2]), zero);
      }
      Dr[j] = csel(ok, vd[j + 1], zero);
    }
    const int64_t K = J + M;
    if constexpr (SRC == SRC_EXPL)
      bK = csel(row_in<IN>(K, n), vb[M + 1], zero);
    else
      bK = csel(row_in<IN>(K, n), cconj(vc[M]), zero);
    first_state = last_state = zero;
  } else if constexpr (cn_src(SRC)) {
    constexpr bool WA = SRC == SRC_CNW;
    CnRaw<M, true, WA> raw;
    cn_fetch<M, true, IN, WA>(A, G, w0, lane, raw);
    cn_build<M, W, PH, true, IN, WA>(A, G, buf, w0, J, lane, wave, raw, Ar, Br, Cr, Dr, bK,
                                     first_state, last_state, ayn);
  } else {  // SRC_SLOTS: row k of the reduced system = U slot of tile k + D slot of tile k-1
    const cd zero = czero();
    auto ld = [](const cd* p) {
      if constexpr (CL)
        return ld_coh(p);
      else
        return *p;
    };
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t r = J + j;
      const bool ok = r < n;
      const int64_t g = G.base + (ok ? r : n - 1);
      const int64_t gp = (ok && r > 0) ? g - 1 : g;
      const cd ua = ld(A.sU + 3 * g), uc = ld(A.sU + 3 * g + 1), ud = ld(A.sU + 3 * g + 2);
      const cd db = ld(A.sD + 3 * gp), da = ld(A.sD + 3 * gp + 1), dd = ld(A.sD + 3 * gp + 2);
      const bool hasp = ok && r > 0;
      Ar[j] = csel(ok, cadd(ua, csel(hasp, da, zero)), mk(1.0, 0.0));
      Br[j] = csel(hasp, db, zero);
      Cr[j] = csel(ok && r < n - 1, uc, zero);
      Dr[j] = csel(ok, cadd(ud, csel(hasp, dd, zero)), zero);
      if (A.ud_halo) {
        const cd h = ld(A.ud_halo + 2 * gp + 1);
        const double kap = cn_kappa(A.dt, A.dxs ? A.dxs[G.sys] : A.dx);
        Dr[j] = cadd(Dr[j], csel(hasp, mk(-kap * h.y, kap * h.x), zero));
      }
    }
    const int64_t K = J + M;
    const int64_t gk = G.base + (K < n ? K - 1 : 0);
    const cd t = ld(A.sD + 3 * gk);
    bK = csel(K < n, t, zero);
    first_state = last_state = zero;
  }
}

template <int W>
struct Log2 {
  static constexpr int v = (W <= 1) ? 0 : 1 + Log2<W / 2>::v;
};
template <>
struct Log2<1> {
  static constexpr int v = 0;
};

template <int M, int W>
struct TileSmem;

template <int M, int W, int SRC, bool IN>
__device__ __forceinline__ void store_tile(const KArgs& A, const Geo& G, TileSmem<M, W>& sm,
                                           cd* buf, int64_t w0, int lane, int wave,
                                           const cd (&x)[M]);

template <int M, int W>
struct TileSmem {
  // Partial blocks left by the nesting levels inside each wavefront (64 / W per wavefront) and,
  // on the way down, psi at their two joint lines: kept in the idle tail of each staging buffer
  // (after the tree nodes and, for M = 8, the diagonals) when they fit there.
  static constexpr int kPer = 64 / W;
  static constexpr size_t kOff = sizeof(Node) * 64 + (M == 8 ? sizeof(double) * 64 * M : 0);
  static constexpr bool kInStage =
      W > 1 && kOff + sizeof(Blk) * kPer <= sizeof(cd) * Stage<M>::QS;
  cd lds[W][Stage<M>::QS];  // per-wavefront staging buffer; holds the tree nodes in between
  Blk xblk[(W > 1 && !kInStage) ? 64 : 1];
  Node xnode[64];
  double wsum[W];
  cd wedge[W];  // PH_FUSE: last new-state row of every wavefront
  __device__ __forceinline__ Blk* part(int w, int k) {
    if constexpr (kInStage)
      return reinterpret_cast<Blk*>(reinterpret_cast<char*>(lds[w]) + kOff) + k;
    else
      return &xblk[w * kPer + k];
  }
};

__device__ __forceinline__ double wave_sum(double v) {
  v += xmove<1>(v);
  v += xmove<2>(v);
  v += xmove<4>(v);
  v += xmove<8>(v);
  v += xmove<16>(v);
  v += xmove<32>(v);
  return v;  // every lane holds the sum, added in the same order
}

// Coalesced store of the tile's solution through the LDS buffer; for the CN source the adjoint
// accumulation (see KArgs) runs on the same coalesced rows.
template <int M, int W, int SRC, bool IN>
__device__ __forceinline__ void store_tile(const KArgs& A, const Geo& G, TileSmem<M, W>& sm,
                                           cd* buf, int64_t w0, int lane, int wave,
                                           const cd (&x)[M]) {
  using S = Stage<M>;
  wave_sync();
#pragma unroll
  for (int j = 0; j < M; ++j) buf[S::addr(lane * M + j + 1)] = x[j];
  wave_sync();
  cd* g = A.x + G.base;
  const bool acc = cn_src(SRC) && A.acc_pa != nullptr;
  double part = 0.0;
  // recompute the row addresses here instead of keeping those of the loads alive across the
  // whole tile (the empty asm hides that they are equal)
  int sl = lane;
  asm volatile("" : "+v"(sl));
  if (!acc) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const int64_t r = w0 + 64 * k + sl;
      if (row_in<IN>(r, G.n)) g[r * G.es] = buf[S::addr(1 + 64 * k + sl)];
    }
  } else {
    // all loads of the tile's rows first: the stores below may alias them as far as the
    // compiler knows, which would otherwise cost one memory round trip per row
    // in two halves of the lane's rows, which keeps the gathered operands within the
    // registers the solve needed
    constexpr int CH = M >= 8 ? M / 2 : M;
#pragma unroll
    for (int c = 0; c < M; c += CH) {
      cd s[CH], ov[CH];
      double dv[CH], xv[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int64_t r = w0 + 64 * (c + k) + sl;
        const int64_t e = G.base + r * G.es;
        cd sk = czero(), o = czero();
        double d0 = 0.0, x0 = 0.0;
        if (row_in<IN>(r, G.n)) {
          sk = cadd(A.acc_pa[e], A.acc_pb[e]);
          if (A.acc_dV) d0 = A.acc_dV[e];
          if (A.xg) x0 = A.xg[e];
          if (A.acc_half) o = g[r * G.es];
        }
        s[k] = sk;
        ov[k] = o;
        dv[k] = d0;
        xv[k] = x0;
      }
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int64_t r = w0 + 64 * (c + k) + sl;
        if (row_in<IN>(r, G.n)) {
          const cd v = buf[S::addr(1 + 64 * (c + k) + sl)];
          const int64_t e = G.base + r * G.es;
          g[r * G.es] = v;
          const cd lam =
              csel(A.acc_half != 0, mk(0.5 * (v.x + ov[k].x), 0.5 * (v.y + ov[k].y)), v);
          const double q = A.acc_tau * (lam.x * s[k].y - lam.y * s[k].x);
          if (A.acc_dV) A.acc_dV[e] = dv[k] + A.vscale * q;
          if (A.xg) part = fma(xv[k], q, part);
        }
      }
    }
  }
  if (acc && A.acc_part) {
    part = wave_sum(part);
    if (lane == 0) sm.wsum[wave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < W; ++w) t += sm.wsum[w];
      A.acc_part[G.gt] = t;
    }
    __syncthreads();
  }
}

template <int M, int W, int SRC, int PH, bool IN>
__device__ __forceinline__ void tile_finish(const KArgs& A, const Geo& G, TileSmem<M, W>& sm,
                                            cd* buf, int64_t w0, int64_t J, int lane, int wave,
                                            cd (&Ar)[M], cd (&Br)[M], cd (&Cr)[M], cd (&Dr)[M],
                                            cd bK, cd fst, cd lst, const double* ayn);

// One tile of T = 64*W*M rows of one system, run by every thread of the workgroup.
//   PH_SINGLE  the tile holds the whole system: RS on its two joint lines, then SS
//   PH_REDUCE  writes the tile's U/D slots at index G.gt of oU/oD (and, for the CN source,
//              its first and last state row to halo_out)
//   PH_SUBST   takes psi at the tile's joint lines from psi_if[G.gt], psi_if[G.gt + 1]
template <int M, int W, int SRC, int PH>
__device__ __forceinline__ void tile_run(const KArgs& A, const Geo& G, TileSmem<M, W>& sm) {
  constexpr int64_t T = 64 * W * M;
  static_assert(sizeof(cd) * Stage<M>::QS >= sizeof(Node) * 64, "node slots fit the stage buffer");

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t t0 = G.tile * T;
  const int64_t w0 = t0 + (int64_t)wave * 64 * M;
  const int64_t J = w0 + (int64_t)lane * M;
  cd* buf = sm.lds[wave];

  cd Ar[M], Br[M], Cr[M], Dr[M], bK, fst, lst;
  constexpr int PL = (PH == PH_FUSE) ? PH_SUBST : PH;  // the rows are those of a PH_SUBST pass
  // PH_FUSE: diagonal of the next step, from this pass's loads of V and xgrid (imaginary parts)
  double ayn[M];
  double* ayp = (PH == PH_FUSE) ? ayn : nullptr;
  // wavefront-uniform choice between the interior path and the general one
  if (SRC != SRC_SLOTS && w0 >= 1 && G.n >= w0 + 64 * M + 1) {
    load_rows<M, W, SRC, PL, true>(A, G, buf, w0, J, lane, wave, Ar, Br, Cr, Dr, bK, fst, lst,
                                   ayp);
    tile_finish<M, W, SRC, PH, true>(A, G, sm, buf, w0, J, lane, wave, Ar, Br, Cr, Dr, bK, fst,
                                     lst, ayp);
  } else {
    load_rows<M, W, SRC, PL, false>(A, G, buf, w0, J, lane, wave, Ar, Br, Cr, Dr, bK, fst, lst,
                                    ayp);
    tile_finish<M, W, SRC, PH, false>(A, G, sm, buf, w0, J, lane, wave, Ar, Br, Cr, Dr, bK, fst,
                                      lst, ayp);
  }
}

// Everything after the rows of the tile are assembled up to SS: level-1 sweeps, nesting, top,
// substitution.  wnode holds this wavefront's 64 tree nodes; sm provides the partial blocks and
// the nodes (xnode) of the levels across wavefronts.  For PH != PH_REDUCE, xo returns this lane's rows J .. J+M-1.
// Crank-Nicolson tiles of M = 8 rows per lane that substitute take reduce_block_rd /
// ss_block_rd (fewer registers, so two 512-lane workgroups fit a CU; with fewer rows per lane
// the extra arithmetic buys no occupancy): keep holds 64 * M doubles of this wavefront's LDS for
// the diagonals between the two, and kap is the off-diagonal magnitude (tau / (2 dx^2)) that
// ss_block_rd recomputes the couplings from.  With an absorbing potential the diagonal's real
// parts (1 + tau W) stay in registers between the two (the staging buffer has no room for them).
// A store that reaches the level of the memory system shared by all XCDs (a relaxed atomic at
// device scope), used for the values a tile hands to the next level: the last workgroup of a
// pass that solves the reduced system itself reads them right after the other workgroups have
// counted themselves done, without a write-back of their L2.
__device__ __forceinline__ void st_coh(cd* p, cd v) {
  __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct NoMid {
  __device__ void operator()(cd&, cd&) const {}
};

template <int M, int W, int SRC, int PH>
struct RdSubst {
  static constexpr bool on = cn_src(SRC) && PH != PH_REDUCE && M == 8;
};

// COH: the slots and edge rows of a PH_REDUCE part are stored device-coherent (st_coh), for a
// fused pass whose last workgroup solves the reduced system (fuse_reduced_last).
// PH_RES: the hand-over of PH_REDUCE, then mid(pJ, pM) (run by the whole workgroup: it waits
// until every tile's slots are in, solves the reduced system and returns psi at the tile's two
// joint lines), then the substitution of PH_SUBST.
template <int M, int W, int SRC, int PH, bool IN, bool RDR = false, bool COH = false, typename SM,
          typename Mid = NoMid>
__device__ __forceinline__ void tile_core(const KArgs& A, const Geo& G, SM& sm, Node* wnode,
                                          double* keep, double kap, int64_t J, int lane, int wave,
                                          cd (&Ar)[M], cd (&Br)[M], cd (&Cr)[M], cd (&Dr)[M],
                                          cd bK, cd fst, cd lst, cd (&xo)[M],
                                          cd* pM_out = nullptr, const Mid& mid = Mid{}) {
  constexpr bool HAND = PH == PH_REDUCE || PH == PH_RES;  // the tile hands its slots over
  constexpr int LW = Log2<W>::v;
  // RDR: a Crank-Nicolson first pass reduced in the RD form as well (fewer registers)
  constexpr bool RD = RdSubst<M, W, SRC, PH>::on || RDR;
  auto put = [](cd* p, cd v) {
    if constexpr (COH)
      st_coh(p, v);
    else
      *p = v;
  };
  if constexpr (HAND && cn_src(SRC)) {
    if (A.halo_out) {
      if (wave == 0 && lane == 0) put(A.halo_out + 2 * G.gt, fst);
      if (wave == W - 1 && lane == 63) put(A.halo_out + 2 * G.gt + 1, lst);
    }
  }

  Blk blk;
  const CnEdges<IN> edges{J, G.n, kap};
  // SRC_CNW: real parts of the diagonal (1 + tau W), held from the reduction to the substitution
  constexpr bool CR = SRC == SRC_CNW;
  double ar[M];
  wave_sync();
  if constexpr (RD) {
    double ay[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      ay[j] = Ar[j].y;
      ar[j] = CR ? Ar[j].x : 1.0;
    }
    if constexpr (PH != PH_REDUCE) {
#pragma unroll
      for (int j = 1; j < M; ++j) keep[j * 64 + lane] = ay[j];
    }
    reduce_block_rd_g<M, CR>(ar, ay, edges, Dr, bK.y, blk);
  } else {
    reduce_block<M, cn_src(SRC)>(Ar, Br, Cr, Dr, bK, blk);
  }
  if constexpr (W == 1) {
    tree_up<6>(blk, wnode, lane);
  } else {
    // The 64 W lane blocks of the tile are nested in 6 + log2 W binary levels.  The lowest
    // log2 W run inside every wavefront and leave 64 / W partial blocks each (lanes 0, W, 2W..);
    // wavefront 0 takes the resulting 64 blocks through the remaining six.  Same critical
    // path as six levels per wavefront followed by log2 W across them, but W log2 W + 6
    // wavefront-levels of work instead of 6 W + log2 W.
    tree_up<LW>(blk, wnode, lane);
    if ((lane & (W - 1)) == 0) *sm.part(wave, lane >> LW) = blk;
    __syncthreads();
    if (wave == 0) {
      blk = *sm.part(lane >> (6 - LW), lane & (64 / W - 1));
      tree_up<6>(blk, sm.xnode, lane);
    }
  }

  cd pJ = czero(), pM = czero();
  if (wave == 0 && lane == 0) {
    if constexpr (HAND) {
      put(A.oU + 3 * G.gt, blk.UA);
      put(A.oU + 3 * G.gt + 1, blk.UC);
      put(A.oU + 3 * G.gt + 2, blk.UD);
      put(A.oD + 3 * G.gt, blk.DB);
      put(A.oD + 3 * G.gt + 1, blk.DA);
      put(A.oD + 3 * G.gt + 2, blk.DD);
    } else if constexpr (PH == PH_SINGLE) {
      // RS on the two joint lines of the tile (the bottom one lies past the system end)
      cd ia0 = crecip(blk.UA);
      cd r = cneg(cmul(blk.DB, ia0));
      cd aT = cfma(r, blk.UC, cadd(mk(1.0, 0.0), blk.DA));
      cd dT = cfma(r, blk.UD, blk.DD);
      pM = cmul(dT, crecip(aT));
      pJ = cmul(cfms(blk.UC, pM, blk.UD), ia0);
    } else {
      pJ = A.psi_if[G.gt];
      const cd nxt = A.psi_if[(G.tile + 1 < G.ntile) ? G.gt + 1 : G.gt];
      pM = csel(G.tile + 1 < G.ntile, nxt, czero());
    }
  }
  if constexpr (PH == PH_RES) mid(pJ, pM);
  if constexpr (PH != PH_REDUCE) {
    if constexpr (W == 1) {
      tree_down<6>(pJ, pM, wnode, lane);
    } else {
      if (wave == 0) {
        tree_down<6>(pJ, pM, sm.xnode, lane);
        cd* q = reinterpret_cast<cd*>(sm.part(lane >> (6 - LW), lane & (64 / W - 1)));
        q[0] = pJ;
        q[1] = pM;
      }
      __syncthreads();
      // every lane reads the pair of its group; the leading lanes' copies start the levels
      const cd* q = reinterpret_cast<const cd*>(sm.part(wave, lane >> LW));
      pJ = q[0];
      pM = q[1];
      tree_down<LW>(pJ, pM, wnode, lane);
    }
    if (pM_out) *pM_out = pM;
    if constexpr (RD) {
      double ay[M];
      ay[0] = 0.0;
#pragma unroll
      for (int j = 1; j < M; ++j) ay[j] = keep[j * 64 + lane];
      ss_block_rd_g<M, CR>(ar, ay, edges, Dr, pJ, pM, xo);
    } else {
      ss_block<M>(Br, Cr, Dr, pJ, pM, xo);
    }
  }
}

// Raises the status flag when a row of this lane is not finite.
template <int M, bool IN>
__device__ __forceinline__ void check_rows(const KArgs& A, const Geo& G, int64_t J, int lane,
                                           const cd (&xo)[M]) {
  bool bad = false;
#pragma unroll
  for (int j = 0; j < M; ++j) bad |= row_in<IN>(J + j, G.n) && !cfinite(xo[j]);
  if (__any(bad) && lane == 0) atomicOr(A.status, 1);
}

// PH_FUSE, after the tile's new state is stored: the rows of the next step (field E_next) from
// that state, reduced as in PH_REDUCE.  The stores left this wavefront's new rows in its staging
// buffer; the rows around them come from the neighbouring wavefronts (their last row through
// wedge) and from the joint line below the lane (pM).  Wavefront 0 has no left neighbour in the
// tile: its joint row takes the explicit half-step without psi_{J-1}, whose term the reduced
// system adds (KArgs::ud_halo); at the start of a system that neighbour is zero anyway.
// STAGED: the rows xo are already in the staging buffer (left there by store_tile); otherwise
// they are put there first.
template <int M, int W, bool IN, int SRC = SRC_CN, bool STAGED = true>
__device__ __forceinline__ void next_rows(const KArgs& A, const Geo& G, TileSmem<M, W>& sm,
                                          cd* buf, int64_t J, int lane, int wave,
                                          const cd (&xo)[M], cd pM, const double* ayn,
                                          const double* arn, double kap, cd (&Ar)[M],
                                          cd (&Br)[M], cd (&Cr)[M], cd (&Dr)[M], cd& bK,
                                          cd& fst, cd& lst) {
  static_assert(M >= 2, "the next step is reduced in the RD form");
  constexpr bool WA = SRC == SRC_CNW;
  using S = Stage<M>;
  if constexpr (!STAGED) {
    wave_sync();
#pragma unroll
    for (int j = 0; j < M; ++j) buf[S::addr(lane * M + j + 1)] = xo[j];
  }
  if (lane == 63) sm.wedge[wave] = xo[M - 1];
  __syncthreads();
  if (lane == 0) buf[S::addr(0)] = csel(wave > 0, sm.wedge[wave > 0 ? wave - 1 : 0], czero());
  if (lane == 63) buf[S::addr(S::QN - 1)] = pM;
  wave_sync();
  cd vp[M + 2];
  stage_read<M>(buf, lane, vp);
  if constexpr (!IN) {
    // rows past the end of the system hold no state
#pragma unroll
    for (int j = 0; j < M + 2; ++j) vp[j] = csel(J - 1 + j < G.n, vp[j], czero());
  }
  wave_sync();
  // the rows of the next step: its diagonal's imaginary parts are ayn (SRC_CNW: the real parts
  // arn = 1 + tau W are this step's), the right-hand side is the explicit half-step of cn_rows
  // with the same diagonal
  const cd zero = czero();
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double w = ayn[j];
    const cd p = vp[j + 1];
    const cd s2 = cadd(vp[j], vp[j + 2]);
    const bool ok = row_in<IN>(J + j, G.n);
    Br[j] = Cr[j] = zero;  // the RD form takes the couplings from kap
    if constexpr (WA) {
      // tau W recovered from 1 + tau W exactly (Sterbenz): the diagonal is this step's to the
      // bit, the explicit side's tau W within an ulp of 1 of it
      const double tw = arn[j] - 1.0;
      Ar[j] = mk(arn[j], w);
      Dr[j] = csel(ok, mk(fma(-tw, p.x, fma(w, p.y, fma(-kap, s2.y, p.x))),
                          fma(-tw, p.y, fma(-w, p.x, fma(kap, s2.x, p.y)))), zero);
    } else {
      Ar[j] = mk(1.0, w);
      Dr[j] = csel(ok, mk(fma(w, p.y, fma(-kap, s2.y, p.x)), fma(-w, p.x, fma(kap, s2.x, p.y))),
                   zero);
    }
  }
  bK = mk(0.0, row_in<IN>(J + M, G.n) ? -kap : 0.0);
  fst = vp[1];
  lst = vp[M];
}

template <int M, int W, bool IN, int SRC = SRC_CN>
__device__ __forceinline__ void fuse_next(const KArgs& A, const Geo& G, TileSmem<M, W>& sm,
                                          cd* buf, int64_t J, int lane, int wave,
                                          const cd (&xo)[M], cd pM, const double* ayn,
                                          const double* arn = nullptr) {
  const double dx = A.dxs ? A.dxs[G.sys] : A.dx;
  const double kap = cn_kappa(A.dt, dx);
  cd Ar[M], Br[M], Cr[M], Dr[M], dummy[M], bK, fst, lst;
  next_rows<M, W, IN, SRC>(A, G, sm, buf, J, lane, wave, xo, pM, ayn, arn, kap, Ar, Br, Cr, Dr,
                           bK, fst, lst);
  Node* wnode = reinterpret_cast<Node*>(buf);
  double* keep = reinterpret_cast<double*>(wnode + 64);
  // reduced in the RD form: the diagonal and the right-hand side are all it keeps per row
  tile_core<M, W, SRC, PH_REDUCE, IN, true, true>(A, G, sm, wnode, keep, kap, J, lane, wave, Ar,
                                                  Br, Cr, Dr, bK, fst, lst, dummy);
}

// Everything after the rows of the tile are assembled: level-1 sweeps, nesting, top, SS, store.
template <int M, int W, int SRC, int PH, bool IN>
__device__ __forceinline__ void tile_finish(const KArgs& A, const Geo& G, TileSmem<M, W>& sm,
                                            cd* buf, int64_t w0, int64_t J, int lane, int wave,
                                            cd (&Ar)[M], cd (&Br)[M], cd (&Cr)[M], cd (&Dr)[M],
                                            cd bK, cd fst, cd lst, const double* ayn) {
  // the staging buffer is idle between the loads and the stores: it holds the nodes and, for
  // substitution along the RD rows, the diagonals after them
  constexpr int PS = (PH == PH_FUSE) ? PH_SUBST : PH;  // the solve that ends in this pass
  Node* wnode = reinterpret_cast<Node*>(buf);
  double* keep = reinterpret_cast<double*>(wnode + 64);
  static_assert(!RdSubst<M, W, SRC, PS>::on ||
                    sizeof(Node) * 64 + sizeof(double) * 64 * M <= sizeof(cd) * Stage<M>::QS,
                "nodes and diagonals fit the stage buffer");
  double kap = 0.0;
  if constexpr (RdSubst<M, W, SRC, PS>::on) {
    const double dx = A.dxs ? A.dxs[G.sys] : A.dx;
    kap = cn_kappa(A.dt, dx);
  }
  cd xo[M];
  cd pM = czero();
  // PH_FUSE with an absorbing potential: the diagonal's real parts for the next step
  constexpr bool KR = PH == PH_FUSE && SRC == SRC_CNW;
  double arn[KR ? M : 1];
  if constexpr (KR) {
#pragma unroll
    for (int j = 0; j < M; ++j) arn[j] = Ar[j].x;
  }
  tile_core<M, W, SRC, PS, IN>(A, G, sm, wnode, keep, kap, J, lane, wave, Ar, Br, Cr, Dr, bK, fst,
                               lst, xo, PH == PH_FUSE ? &pM : nullptr);
  if constexpr (PS != PH_REDUCE) {
    check_rows<M, IN>(A, G, J, lane, xo);
    if constexpr (SRC == SRC_SLOTS) {
#pragma unroll
      for (int j = 0; j < M; ++j)
        if (J + j < G.n) A.x[G.base + J + j] = xo[j];
    } else {
      store_tile<M, W, SRC, IN>(A, G, sm, buf, w0, lane, wave, xo);
    }
  }
  if constexpr (PH == PH_FUSE && cn_src(SRC))
    fuse_next<M, W, IN, SRC>(A, G, sm, buf, J, lane, wave, xo, pM, ayn, KR ? arn : nullptr);
}

// Waves per SIMD that the register allocation of a tile kernel must allow: the fused pass of
// 8 rows per lane carries the next step's diagonal through its first half and sits one
// register above the budget of 3 wavefronts; the others keep the compiler's choice.
template <int M, int PH, int SRC = SRC_CN>
constexpr int tile_min_waves() {
  return (PH == PH_FUSE && M == 8 && cn_src(SRC)) ? 3 : 1;
}

// The reduced system of a PH_FUSE pass over one system, solved in the same launch: every
// workgroup waits until its own stores of slots and edge rows (device-coherent, fuse_next) have
// completed and counts itself done; the last one to do so reads them after an acquire at device
// scope and solves the system on the K <= 128 W tile joints as one whole-system tile of 2 rows
// per lane (the deferred joint-row terms from the new edge rows, as the separate launch would),
// writing psi at the joints where the next pass reads it.  Nobody waits on anybody, and the
// pass's own reads of psi at the joints happened before its workgroups counted themselves.
template <int M, int W>
__device__ __forceinline__ void fuse_reduced_last(const KArgs& A, TileSmem<M, W>& sm, int& last) {
  static_assert(sizeof(TileSmem<2, W>) <= sizeof(TileSmem<M, W>), "LDS of the reduced solve");
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);  // this wavefront's stores have completed
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nwg = (int)(gridDim.x * gridDim.y);
    const int done = atomicAdd(A.inl_sync, 1);
    last = done == nwg - 1;
    if (last) atomicExch(A.inl_sync, 0);  // every workgroup has counted: ready for the next pass
  }
  __syncthreads();
  if (!last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  KArgs B = A;
  B.sU = A.oU;
  B.sD = A.oD;
  B.ud_halo = A.halo_out;
  B.x = const_cast<cd*>(A.psi_if);
  B.rhs = nullptr;
  Geo G;
  G.sys = 0;
  G.tile = 0;
  G.n = A.ntiles;
  G.base = 0;
  G.cbase = 0;
  G.es = 1;
  G.gt = 0;
  G.ntile = 1;
  tile_run<2, W, SRC_SLOTS, PH_SINGLE>(B, G, *reinterpret_cast<TileSmem<2, W>*>(&sm));
}

// One workgroup = one tile of T = 64*W*M rows of one system.
template <int M, int W, int SRC, int PH>
__global__ __launch_bounds__(64 * W, (tile_min_waves<M, PH, SRC>())) void k_tile(KArgs A) {
  __shared__ TileSmem<M, W> sm;
  const Geo G = geometry<PH>(A);
  tile_run<M, W, SRC, PH>(A, G, sm);
  if constexpr (PH == PH_FUSE && cn_src(SRC)) {
    __shared__ int last;
    if (A.inl_sync) fuse_reduced_last<M, W>(A, sm, last);
  }
}

// ------------------------------------------------------- chunked first-level partitions
// First-level partitions larger than one workgroup's tile (8192 and 16384 rows: C = 2 or 4
// chunks of T = 4096 rows, 8 rows per lane, 8 wavefronts) for the solve of explicit a, b, c, d.
// PH_REDUCE: the workgroup reduces the chunks of its partition one after the other (as k_tile),
// keeps their slots in LDS and merges them (the block merge of the nesting levels) into the
// partition's two slots.  PH_SUBST: it reduces the chunks again, solves for psi at the chunk
// joints from the merged blocks and the partition's own joint values, and substitutes chunk by
// chunk, which reads each chunk's rows a third time: a partition whose rows do not fit one
// workgroup's registers costs one more pass over the matrix.
template <int C>
struct ChunkSmem {
  TileSmem<8, 8> t;
  cd cU[3 * C], cD[3 * C];  // the chunks' slots
  cd cpsi[C + 1];           // psi at the chunk joints and at the partition's end
  Node nodes[C];            // chunk joint c eliminated in the merge of chunks 0 .. c
};

template <int C, int PH>
__global__ __launch_bounds__(512) void k_tile_chunk(KArgs A) {
  constexpr int M = 8, W = 8;
  constexpr int64_t T = 64 * W * M;
  static_assert(PH == PH_REDUCE || PH == PH_SUBST, "two-pass partitions");
  __shared__ ChunkSmem<C> sm;
  const Geo P = geometry<PH>(A);  // the partition: tile = its index in the system, gt its slots
  KArgs B = A;
  B.oU = sm.cU;
  B.oD = sm.cD;
  // the partition's rows as a system of their own from the partition's first row (rows past its
  // end, up to the end of the system, are read as the chunks' neighbours)
  Geo G = P;
  const int64_t r0 = P.tile * C * T;
  G.base = P.base + r0 * P.es;
  G.cbase = P.cbase + r0 * P.es;
  G.n = P.n - r0;
  G.ntile = C;
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    G.tile = c;
    G.gt = c;
    tile_run<M, W, SRC_EXPL, PH_REDUCE>(B, G, sm.t);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    auto blk = [&](int c) {
      Blk b;
      b.UA = sm.cU[3 * c];
      b.UC = sm.cU[3 * c + 1];
      b.UD = sm.cU[3 * c + 2];
      b.DB = sm.cD[3 * c];
      b.DA = sm.cD[3 * c + 1];
      b.DD = sm.cD[3 * c + 2];
      return b;
    };
    Blk b = blk(0);
    for (int c = 1; c < C; ++c) merge_into(b, blk(c), sm.nodes[c]);
    if constexpr (PH == PH_REDUCE) {
      A.oU[3 * P.gt] = b.UA;
      A.oU[3 * P.gt + 1] = b.UC;
      A.oU[3 * P.gt + 2] = b.UD;
      A.oD[3 * P.gt] = b.DB;
      A.oD[3 * P.gt + 1] = b.DA;
      A.oD[3 * P.gt + 2] = b.DD;
    } else {
      const cd pJ = A.psi_if[P.gt];
      const cd pM = P.tile + 1 < P.ntile ? A.psi_if[P.gt + 1] : czero();
      sm.cpsi[0] = pJ;
      sm.cpsi[C] = pM;
      cd nx = pM;
      for (int c = C - 1; c >= 1; --c) {
        const Node t = sm.nodes[c];
        nx = cfms(t.C, nx, cfms(t.B, pJ, t.dl));
        sm.cpsi[c] = nx;
      }
    }
  }
  if constexpr (PH == PH_SUBST) {
    __syncthreads();
    B.psi_if = sm.cpsi;
    G.ntile = C + 1;  // every chunk reads psi at its end joint from cpsi
#pragma unroll 1
    for (int c = 0; c < C; ++c) {
      G.tile = c;
      G.gt = c;
      tile_run<M, W, SRC_EXPL, PH_SUBST>(B, G, sm.t);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ resident propagation
// Every step of a Crank-Nicolson propagation of one system in one launch.  Workgroup t owns
// tile t for the whole sequence and keeps its rows in registers: the right-hand side of the RD
// rows (Table 1 with substitution along them), and per row the two terms of the diagonal's
// imaginary part (with an absorbing potential also its real part, 1 + tau W), so that after the
// first loads a step neither reads nor writes the state in memory.  Per step the
// tile reduces its rows, nested inside the tile as in k_tile, stores its two slots and edge rows
// device-coherently and raises its flag; every workgroup waits (bounded poll) until all K flags
// show the step, then solves the reduced system on the K tile joints itself (a whole-system
// tile of 2 rows per lane in its own LDS, the deferred left-neighbour terms added from the edge
// rows as in the chained passes), keeps psi at its own two joints, substitutes (SS) and builds
// the next step's rows from the new state in registers (next_rows).  Slots and edge rows
// alternate between two buffers by step parity: a tile publishes step k+1 only after every tile
// has published step k, so after every tile has read step k-1's values.  The state is written
// once, after the last step.
struct ResArgs {
  const double* E;  // field per step (device, nsteps values), or null for a zero field
  int nsteps;
  int* flags;       // one per tile: steps published in this launch; zero between launches
  int* sync;        // [-, -, abort, workgroups out]; zero between launches
  int spin;         // polls before a wait gives up (sets abort and status bit 4)
  int64_t bufstep;  // elements between the two parity buffers of oU, oD (3 K) and halo (2 K)
  cd* ckpt;         // states before the steps k = K, 2K, ... at ckpt + (k / K) n, or null (the
  int K;            // state before step 0 is the caller's copy)
};

template <int M, int W>
struct ResSmem {
  TileSmem<M, W> t;
  TileSmem<2, W> r;  // the reduced solve
  cd pj, pm;         // psi at this tile's joint lines
  int flag;          // broadcast: 2 aborted, 1 last workgroup out
};

// The step's hand-over and reduced solve; returns false when the launch aborted.
template <int M, int W>
__device__ __forceinline__ bool res_exchange(const KArgs& A, const ResArgs& R, ResSmem<M, W>& sm,
                                             int k, cd& pJ, cd& pM) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int K = (int)A.ntiles;
  const int t = (int)blockIdx.x;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);  // this wavefront's slot and edge-row stores have completed
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (wave == 0) {
    if (lane == 0) __hip_atomic_store(R.flags + t, k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int out = 0;
    for (int it = 0;; ++it) {
      bool in = true;
      for (int i = lane; i < K; i += 64)
        in &= __hip_atomic_load(R.flags + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > k;
      if (__all(in)) break;
      const bool ab = __hip_atomic_load(R.sync + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (it >= R.spin || __any(ab)) {  // (wavefront-uniform)
        if (lane == 0) {
          atomicExch(R.sync + 2, 1);
          atomicOr(A.status, 4);
        }
        out = 2;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) sm.flag = out;
  }
  __syncthreads();
  if (sm.flag == 2) return false;
  // the reduced system on the tile joints, in this workgroup (its values read device-coherent)
  KArgs B = A;
  B.sU = A.oU;
  B.sD = A.oD;
  B.ud_halo = k > 0 ? A.halo_out : nullptr;  // step 0's rows took both neighbours from memory
  B.rhs = nullptr;
  B.dxs = nullptr;
  Geo G;
  G.sys = 0;
  G.tile = 0;
  G.n = K;
  G.base = 0;
  G.cbase = 0;
  G.es = 1;
  G.gt = 0;
  G.ntile = 1;
  {
    const int64_t w0 = (int64_t)wave * 64 * 2;
    const int64_t J = w0 + (int64_t)lane * 2;
    cd* buf = sm.r.lds[wave];
    cd Ar[2], Br[2], Cr[2], Dr[2], bK, fst, lst, xo[2];
    load_rows<2, W, SRC_SLOTS, PH_SINGLE, false, true>(B, G, buf, w0, J, lane, wave, Ar, Br, Cr,
                                                        Dr, bK, fst, lst);
    Node* wnode = reinterpret_cast<Node*>(buf);
    double* keep = reinterpret_cast<double*>(wnode + 64);
    tile_core<2, W, SRC_SLOTS, PH_SINGLE, false>(B, G, sm.r, wnode, keep, 0.0, J, lane, wave, Ar,
                                                 Br, Cr, Dr, bK, fst, lst, xo);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (J + j == t) sm.pj = xo[j];
      if (J + j == t + 1) sm.pm = xo[j];
    }
  }
  __syncthreads();
  pJ = sm.pj;
  pM = t + 1 < K ? sm.pm : czero();
  return true;
}

template <int M, int W, int SRC, bool IN>
__device__ __forceinline__ void resident_run(const KArgs& A, const ResArgs& R, const Geo& G,
                                             ResSmem<M, W>& sm, int64_t w0, int64_t J, int lane,
                                             int wave) {
  constexpr bool WA = SRC == SRC_CNW;
  cd* buf = sm.t.lds[wave];
  cd Ar[M], Br[M], Cr[M], Dr[M], bK, fst, lst;
  double vk[2 * M];     // per row: tau (1/dx^2 + vscale v), then tau x
  double arn[WA ? M : 1];  // SRC_CNW: the diagonal's real parts 1 + tau W, the same every step
  {
    KArgs A0 = A;
    A0.E_mat = A0.E_rhs = R.E ? R.E[0] : 0.0;
    CnRaw<M, true, WA> raw;
    cn_fetch<M, true, IN, WA>(A0, G, w0, lane, raw);
    cn_build<M, W, PH_REDUCE, true, IN, WA>(A0, G, buf, w0, J, lane, wave, raw, Ar, Br, Cr, Dr,
                                            bK, fst, lst, nullptr, vk);
  }
  if constexpr (WA) {
#pragma unroll
    for (int j = 0; j < M; ++j) arn[j] = Ar[j].x;
  }
  const double kap = cn_kappa(A.dt, A.dx);
  bool ok = true;
  for (int k = 0; k < R.nsteps; ++k) {
    KArgs Ak = A;  // this step's parity buffer of slots and edge rows
    const int64_t off = (k & 1) ? R.bufstep : 0;
    Ak.oU = A.oU + 3 * off;
    Ak.oD = A.oD + 3 * off;
    Ak.halo_out = A.halo_out + 2 * off;
    Node* wnode = reinterpret_cast<Node*>(buf);
    double* keep = reinterpret_cast<double*>(wnode + 64);
    cd xo[M];
    cd pM = czero();
    auto mid = [&](cd& pj, cd& pm) { ok = res_exchange<M, W>(Ak, R, sm, k, pj, pm); };
    tile_core<M, W, SRC, PH_RES, IN, true, true>(Ak, G, sm.t, wnode, keep, kap, J, lane, wave, Ar,
                                                 Br, Cr, Dr, bK, fst, lst, xo, &pM, mid);
    if (!ok) return;
    if (k + 1 == R.nsteps) {
      check_rows<M, IN>(A, G, J, lane, xo);
      store_tile<M, W, SRC, IN>(A, G, sm.t, buf, w0, lane, wave, xo);
      return;
    }
    if (R.ckpt && (k + 1) % R.K == 0) {  // the state before step k + 1
      KArgs Ac = A;
      Ac.x = R.ckpt + (int64_t)((k + 1) / R.K) * A.n;
      store_tile<M, W, SRC, IN>(Ac, G, sm.t, buf, w0, lane, wave, xo);
    }
    const double En = R.E ? R.E[k + 1] : 0.0;
    double ayn[M];
#pragma unroll
    for (int j = 0; j < M; ++j) ayn[j] = row_in<IN>(J + j, G.n) ? fma(vk[M + j], En, vk[j]) : 0.0;
    next_rows<M, W, IN, SRC, false>(A, G, sm.t, buf, J, lane, wave, xo, pM, ayn,
                                    WA ? arn : nullptr, kap, Ar, Br, Cr, Dr, bK, fst, lst);
  }
}

// One workgroup per tile of T = 64 W M rows of the one system (A.n rows, A.ntiles <= 128 W
// tiles, unit stride); the host launches it only when every workgroup fits on the GPU at once.
// SRC: SRC_CN, or SRC_CNW for a potential with an absorbing part (A.Wabs, A.wscale).
template <int M, int W, int SRC>
__global__ __launch_bounds__(64 * W) void k_resident(KArgs A, ResArgs R) {
  __shared__ ResSmem<M, W> sm;
  Geo G;
  G.sys = 0;
  G.tile = blockIdx.x;
  G.n = A.n;
  G.base = 0;
  G.cbase = 0;
  G.es = 1;
  G.gt = blockIdx.x;
  G.ntile = A.ntiles;
  constexpr int64_t T = 64 * W * M;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t w0 = G.tile * T + (int64_t)wave * 64 * M;
  const int64_t J = w0 + (int64_t)lane * M;
  if (w0 >= 1 && G.n >= w0 + 64 * M + 1)
    resident_run<M, W, SRC, true>(A, R, G, sm, w0, J, lane, wave);
  else
    resident_run<M, W, SRC, false>(A, R, G, sm, w0, J, lane, wave);
  __syncthreads();
  if (threadIdx.x == 0) sm.flag = atomicAdd(R.sync + 3, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (sm.flag == 1 && wave == 0) {
    // the last workgroup out: flags and words are ready for the next launch
    for (int i = lane; i < (int)A.ntiles; i += 64)
      __hip_atomic_store(R.flags + i, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lane == 0) {
      atomicExch(R.sync + 2, 0);
      atomicExch(R.sync + 3, 0);
    }
  }
}

// ------------------------------------------------------------ several right-hand sides
// One workgroup = one tile of T = 64*W*M rows of ONE matrix (a, b, c shared by the batch:
// cshared) and nrhs right-hand sides of it (systems blockIdx.y * nrhs + r).  The matrix rows
// are loaded once and factored once: the lane blocks' reduction and every nesting level keep
// their pivots' reciprocals and multipliers (BlkFac, NodeFac; Sec. 5.2.4 stores the r factors
// so that most of RD and RU needs no d).  The loop over the right-hand sides then loads only
// d_r and repeats the updates of d, the top of the tile and the substitution: the matrix
// crosses the memory bus once per tile, and no right-hand side pays for a division.
// The current right-hand side's node values (dl) live where the single-right-hand-side kernels
// keep their nodes: at the head of each wavefront's staging buffer, idle between the
// transposition of d and the store, and for the levels across the wavefronts in xnode.
template <int M, int W>
struct MrhsSmem {
  TileSmem<M, W> t;              // staging buffers, partial blocks between levels, node values
  NodeFac wfac[W][64];           // per wavefront: factors of its nesting levels
  NodeFac xfac[W > 1 ? 64 : 1];  // the levels across the wavefronts (wavefront 0)
};

// Rows w0 + 64k + lane (k < M) of one right-hand side, as stage_fetch without the halo rows
// (the substitution needs no neighbours of d).
template <int M, bool IN>
__device__ __forceinline__ void rhs_fetch(const cd* g, int64_t es, int64_t w0, int64_t n,
                                          int lane, cd (&v)[M]) {
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const int64_t r = w0 + 64 * k + lane;
    if constexpr (IN) {
      v[k] = sel(true, g[r * es], czero());
    } else {
      const cd t = g[(r < n ? r : n - 1) * es];
      v[k] = sel(r < n, t, czero());
    }
  }
}

// Right-hand side r of the workgroup (system s0 + r) on the factored tile: its d is in cur
// (fetched two right-hand sides earlier), which then receives the d of right-hand side r + 2.
// Returns false, uniformly across the workgroup, once r is past the workgroup's share.
template <int M, int W, int PH, bool IN>
__device__ __forceinline__ bool mrhs_step(const KArgs& A, const Geo& G0, MrhsSmem<M, W>& sm,
                                          cd* buf, cd* wdl, cd* xdl, const BlkFac<M>& F,
                                          const Blk& top, int64_t w0, int64_t J, int lane,
                                          int wave, int64_t s0, int r, cd (&cur)[M]) {
  constexpr int LW = Log2<W>::v;
  const int64_t n = G0.n;
  const cd one = mk(1.0, 0.0), zero = czero();
  Geo G = G0;
  G.sys = s0 + r;
  if (r >= A.nrhs || G.sys >= A.batch) return false;
  G.base = G.sys * A.bs;
  G.gt = G.sys * A.ntiles + G.tile;
  // psi at the tile's two joint lines, loaded before this right-hand side's elimination so
  // that the top of the tile does not wait for memory
  cd qJ = zero, qM = zero;
  if constexpr (PH == PH_SUBST) {
    qJ = A.psi_if[G.gt];
    qM = A.psi_if[(G.tile + 1 < G.ntile) ? G.gt + 1 : G.gt];
  }
  cd vd[M + 2];
  transpose_in<M>(buf, lane, cur, zero, vd);
  if (r + 2 < A.nrhs && G.sys + 2 < A.batch)
    rhs_fetch<M, IN>(A.d + (G.sys + 2) * A.bs, G.es, w0, n, lane, cur);
  cd Dr[M];
#pragma unroll
  for (int j = 0; j < M; ++j) Dr[j] = csel(row_in<IN>(J + j, n), vd[j + 1], zero);
  cd UD, DD;
  reduce_block_rhs<M>(F, Dr, UD, DD);
  if constexpr (W == 1) {
    tree_up_rhs<6>(UD, DD, sm.wfac[0], wdl, lane);
  } else {
    tree_up_rhs<LW>(UD, DD, sm.wfac[wave], wdl, lane);
    if ((lane & (W - 1)) == 0) {
      Blk* q = sm.t.part(wave, lane >> LW);
      q->UD = UD;
      q->DD = DD;
    }
    __syncthreads();
    if (wave == 0) {
      const Blk* q = sm.t.part(lane >> (6 - LW), lane & (64 / W - 1));
      UD = q->UD;
      DD = q->DD;
      tree_up_rhs<6>(UD, DD, sm.xfac, xdl, lane);
    }
  }
  cd pJ = zero, pM = zero;
  if (wave == 0 && lane == 0) {
    if constexpr (PH == PH_REDUCE) {
      A.oU[3 * G.gt] = top.UA;
      A.oU[3 * G.gt + 1] = top.UC;
      A.oU[3 * G.gt + 2] = UD;
      A.oD[3 * G.gt] = top.DB;
      A.oD[3 * G.gt + 1] = top.DA;
      A.oD[3 * G.gt + 2] = DD;
    } else if constexpr (PH == PH_SINGLE) {
      // RS on the two joint lines of the tile (the bottom one lies past the system end)
      const cd ia0 = crecip(top.UA);
      const cd rr = cneg(cmul(top.DB, ia0));
      const cd aT = cfma(rr, top.UC, cadd(one, top.DA));
      const cd dT = cfma(rr, UD, DD);
      pM = cmul(dT, crecip(aT));
      pJ = cmul(cfms(top.UC, pM, UD), ia0);
    } else {
      pJ = qJ;
      pM = csel(G.tile + 1 < G.ntile, qM, zero);
    }
  }
  if constexpr (PH != PH_REDUCE) {
    if constexpr (W == 1) {
      tree_down_fac<6>(pJ, pM, sm.wfac[0], wdl, lane);
    } else {
      if (wave == 0) {
        tree_down_fac<6>(pJ, pM, sm.xfac, xdl, lane);
        cd* q = reinterpret_cast<cd*>(sm.t.part(lane >> (6 - LW), lane & (64 / W - 1)));
        q[0] = pJ;
        q[1] = pM;
      }
      __syncthreads();
      const cd* q = reinterpret_cast<const cd*>(sm.t.part(wave, lane >> LW));
      pJ = q[0];
      pM = q[1];
      tree_down_fac<LW>(pJ, pM, sm.wfac[wave], wdl, lane);
    }
    cd xo[M];
    ss_block<M>(F.Bt, F.Ct, Dr, pJ, pM, xo);
    check_rows<M, IN>(A, G, J, lane, xo);
    store_tile<M, W, SRC_EXPL, IN>(A, G, sm.t, buf, w0, lane, wave, xo);
  }
  __syncthreads();  // the staging buffers and partial blocks are reused by the next one
  return true;
}

template <int M, int W, int PH, bool IN>
__device__ __forceinline__ void tile_run_mrhs(const KArgs& A, const Geo& G0, MrhsSmem<M, W>& sm,
                                              int64_t w0, int64_t J, int lane, int wave) {
  constexpr int LW = Log2<W>::v;
  const int64_t n = G0.n;
  const cd one = mk(1.0, 0.0), zero = czero();
  cd* buf = sm.t.lds[wave];
  cd* wdl = buf;
  cd* xdl = reinterpret_cast<cd*>(sm.t.xnode);
  static_assert(sizeof(cd) * 64 <= sizeof(Node) * 64, "node values fit the node space");
  BlkFac<M> F;
  Blk top;  // wavefront 0, lane 0: the matrix part of the whole tile's block
  {
    cd va[M + 2], vb[M + 2], vc[M + 2];
    {
      cd ra[M], rb[M], rc[M], ha, hb, hc;
      stage_fetch<M, IN>(A.a + G0.cbase, G0.es, w0, n, lane, one, ra, ha);
      stage_fetch<M, IN>(A.b + G0.cbase, G0.es, w0, n, lane, zero, rb, hb);
      stage_fetch<M, IN>(A.c + G0.cbase, G0.es, w0, n, lane, zero, rc, hc);
      transpose_in<M>(buf, lane, ra, ha, va);
      transpose_in<M>(buf, lane, rb, hb, vb);
      transpose_in<M>(buf, lane, rc, hc, vc);
    }
    cd Ar[M], Br[M], Cr[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t q = J + j;
      const bool ok = row_in<IN>(q, n);
      const bool pos = ok && row_pos<IN>(q), notlast = ok && row_notlast<IN>(q, n);
      Ar[j] = csel(ok, va[j + 1], one);
      Br[j] = csel(pos, vb[j + 1], zero);
      Cr[j] = csel(notlast, vc[j + 1], zero);
    }
    const cd bK = csel(row_in<IN>(J + M, n), vb[M + 1], zero);
    reduce_block_fac<M>(Ar, Br, Cr, bK, F, top);
  }
  if constexpr (W == 1) {
    tree_up_fac<6>(top, sm.wfac[0], lane);
  } else {
    // the same split of the levels as the single right-hand side (tile_core)
    tree_up_fac<LW>(top, sm.wfac[wave], lane);
    if ((lane & (W - 1)) == 0) *sm.t.part(wave, lane >> LW) = top;
    __syncthreads();
    if (wave == 0) {
      top = *sm.t.part(lane >> (6 - LW), lane & (64 / W - 1));
      tree_up_fac<6>(top, sm.xfac, lane);
    }
    __syncthreads();  // the partial blocks' space is the right-hand sides' from here on
  }

  const int64_t s0 = G0.sys * A.nrhs;
  // d of the next two right-hand sides is in flight while one is eliminated: two register
  // buffers, each refilled as soon as its rows are in LDS
  cd rdA[M], rdB[M];
  if (s0 < A.batch) rhs_fetch<M, IN>(A.d + s0 * A.bs, G0.es, w0, n, lane, rdA);
  if (A.nrhs > 1 && s0 + 1 < A.batch)
    rhs_fetch<M, IN>(A.d + (s0 + 1) * A.bs, G0.es, w0, n, lane, rdB);
  for (int r = 0; r < A.nrhs; r += 2) {
    if (!mrhs_step<M, W, PH, IN>(A, G0, sm, buf, wdl, xdl, F, top, w0, J, lane, wave, s0, r, rdA))
      break;
    if (!mrhs_step<M, W, PH, IN>(A, G0, sm, buf, wdl, xdl, F, top, w0, J, lane, wave, s0, r + 1,
                                 rdB))
      break;
  }
}

template <int M, int W, int PH>
__global__ __launch_bounds__(64 * W) void k_tile_mrhs(KArgs A) {
  __shared__ MrhsSmem<M, W> sm;
  const Geo G = geometry<PH>(A);
  constexpr int64_t T = 64 * W * M;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t w0 = G.tile * T + (int64_t)wave * 64 * M;
  const int64_t J = w0 + (int64_t)lane * M;
  if (w0 >= 1 && G.n >= w0 + 64 * M + 1)
    tile_run_mrhs<M, W, PH, true>(A, G, sm, w0, J, lane, wave);
  else
    tile_run_mrhs<M, W, PH, false>(A, G, sm, w0, J, lane, wave);
}

// ------------------------------------------------------------------ interleaved batches
// Uniform batches whose neighbouring systems are neighbours in memory (batch_stride 1, e.g. ADI
// y-lines): the 64 lanes of a wavefront take 64 adjacent systems, so every row is one coalesced
// 1 KiB access.  A workgroup owns a tile of T = W*M rows of those 64 systems; wavefront w holds
// rows w*M .. w*M+M-1 of the tile in each lane (level 1, Table 1 in registers).  Level 2 runs
// down the W joint lines of each system inside one lane: a sequential elimination of joint lines
// 1 .. W-1 (JU/JD on blocks with one interior joint line), every lane busy with its own system.
template <int M, int W>
struct ColSmem {
  Blk blk[W][64];       // level-1 blocks; after the elimination, the node of joint line w
  cd jpsi[W + 1][64];   // psi at the tile's joint lines
  double wpart[W][64];  // adjoint partial sums per wavefront and system
};

// Rows r0-1 .. r0+M of this lane's system, loaded clamped and selected.  The row base
// g + r*es is the same for the whole wavefront (r0 is uniform), the lane adds its byte offset
// bofs: the loads take a scalar base and one 32-bit vector offset, no 64-bit address per row.
template <int M, typename T>
__device__ __forceinline__ void col_fetch(const T* g, uint32_t bofs, int64_t es, int64_t r0,
                                          int64_t n, T fill, T (&v)[M + 2]) {
#pragma unroll
  for (int j = 0; j < M + 2; ++j) {
    const int64_t r = r0 - 1 + j;
    const int64_t rc = r < 0 ? 0 : (r < n ? r : n - 1);
    const T t = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(g + rc * es) + bofs);
    v[j] = sel(r >= 0 && r < n, t, fill);
  }
}

// element (row r) of this lane's system in an interleaved array: scalar row base + lane offset
template <typename T>
__device__ __forceinline__ T& col_at(T* g, uint32_t bofs, int64_t r, int64_t es) {
  typedef typename std::conditional<std::is_const<T>::value, const char, char>::type B;
  return *reinterpret_cast<T*>(reinterpret_cast<B*>(g + r * es) + bofs);
}

template <int M, int W, int SRC, int PH>
__global__ __launch_bounds__(64 * W) void k_cols(KArgs A) {
  __shared__ ColSmem<M, W> sm;
  constexpr int64_t T = (int64_t)W * M;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // consecutive workgroups take neighbouring column groups of the same rows, so the rows that
  // run concurrently are read as long contiguous runs
  const int64_t ncg = (A.batch + 63) / 64;
  int64_t bid = blockIdx.x;
  if constexpr (PH == PH_SUBST) {
    if (A.rev) bid = rev_linear(blockIdx.x, gridDim.x);
  }
  const int64_t cg = bid % ncg;
  const int64_t sys = cg * 64 + lane;
  const bool live = sys < A.batch;
  // the batch stride is 1: system s starts at element s; lanes address their system as the
  // column group's first element plus a byte offset
  const int64_t c0 = cg * 64;
  const uint32_t ob16 = (uint32_t)((live ? lane : A.batch - 1 - c0) * 16);
  const uint32_t ob8 = ob16 / 2;
  Geo G;
  G.sys = live ? sys : A.batch - 1;
  G.n = A.n;
  G.es = A.es;
  G.base = G.sys * A.bs;
  G.cbase = G.base;
  G.tile = bid / ncg;
  G.ntile = A.ntiles;
  G.gt = G.sys * A.ntiles + G.tile;
  const int64_t r0 = G.tile * T + (int64_t)wave * M;
  const int64_t n = G.n;
  const cd zero = czero();
  // a Crank-Nicolson reduce pass keeps nothing for substitution: the forward-sum form of RU
  // (reduce_block_rd) then needs no row of the lane held for a backward sweep
  constexpr bool RDR = SRC == SRC_CN && PH == PH_REDUCE && M >= 2;
  double kap = 0.0;
  cd Ar[M], Br[M], Cr[M], Dr[M], bK, fst = zero, lst = zero;
  if constexpr (SRC == SRC_EXPL || SRC == SRC_EXPL_CT) {
    cd va[M + 2], vb[M + 2], vc[M + 2], vd[M + 2];
    col_fetch<M>(A.a + c0, ob16, G.es, r0, n, mk(1.0, 0.0), va);
    col_fetch<M>(A.b + c0, ob16, G.es, r0, n, zero, vb);
    col_fetch<M>(A.c + c0, ob16, G.es, r0, n, zero, vc);
    col_fetch<M>(A.d + c0, ob16, G.es, r0, n, zero, vd);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t r = r0 + j;
      const bool ok = r < n;
      if constexpr (SRC == SRC_EXPL) {
        Ar[j] = csel(ok, va[j + 1], mk(1.0, 0.0));
        Br[j] = csel(ok && r > 0, vb[j + 1], zero);
        Cr[j] = csel(ok && r < n - 1, vc[j + 1], zero);
      } else {
        Ar[j] = csel(ok, cconj(va[j + 1]), mk(1.0, 0.0));
        Br[j] = csel(ok && r > 0, cconj(vc[j]), zero);
        Cr[j] = csel(ok && r < n - 1, cconj(vb[j + 2]), zero);
      }
      Dr[j] = csel(ok, vd[j + 1], zero);
    }
    if constexpr (SRC == SRC_EXPL)
      bK = csel(r0 + M < n, vb[M + 1], zero);
    else
      bK = csel(r0 + M < n, cconj(vc[M]), zero);
  } else if constexpr (SRC == SRC_LCOUP) {
    // rows l = l0 + r of the field coupling at radial point r_s = (s + 1) dx of this lane's
    // system: off-diagonals i tau E r_s c_l (pure imaginary), diagonal 1
    const double sc = 0.5 * A.dt * A.E_mat * ((double)(G.sys + 1) * A.dx);
    cd vp[M + 2];
    col_fetch<M>(A.psi + c0, ob16, G.es, r0, n, zero, vp);
    if constexpr (PH == PH_SUBST) {
      // the neighbouring tiles' edge rows may already hold the new state
      if (wave == 0 && G.tile > 0) vp[0] = A.halo_in[2 * (G.gt - 1) + 1];
      if (wave == W - 1 && G.tile + 1 < G.ntile) vp[M + 1] = A.halo_in[2 * (G.gt + 1)];
    }
    auto cl = [&](int64_t l) {
      return (double)(l + 1) / sqrt((double)(2 * l + 1) * (double)(2 * l + 3));
    };
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t r = r0 + j;
      const bool ok = r < n;
      const double cb = (ok && r > 0) ? sc * cl(A.l0 + r - 1) : 0.0;
      const double cc = (ok && r < n - 1) ? sc * cl(A.l0 + r) : 0.0;
      Ar[j] = mk(1.0, 0.0);
      Br[j] = mk(0.0, cb);
      Cr[j] = mk(0.0, cc);
      const cd p = vp[j + 1], lo = vp[j], hi = vp[j + 2];
      Dr[j] = csel(ok, mk(p.x + cb * lo.y + cc * hi.y, p.y - cb * lo.x - cc * hi.x), zero);
    }
    bK = mk(0.0, (r0 + M < n) ? sc * cl(A.l0 + r0 + M - 1) : 0.0);
    fst = vp[1];
    lst = vp[M];
  } else {  // SRC_CN
    const double dx = A.dxs ? A.dxs[G.sys] : A.dx;
    const double tau = 0.5 * A.dt;
    const double idx2 = 1.0 / (dx * dx);
    kap = cn_kappa(A.dt, dx);
    const bool given = A.rhs != nullptr;
    cd vp[M + 2];
    double vv[M + 2], xv[M + 2];
    col_fetch<M>((given ? A.rhs : A.psi) + c0, ob16, G.es, r0, n, zero, vp);
    col_fetch<M>(A.V + c0, ob8, G.es, r0, n, 0.0, vv);
    if (A.xg) {
      col_fetch<M>(A.xg + c0, ob8, G.es, r0, n, 0.0, xv);
    } else {
#pragma unroll
      for (int j = 0; j < M + 2; ++j) xv[j] = 0.0;
    }
    if constexpr (PH == PH_SUBST) {
      // the neighbouring tiles' edge rows may already hold the new state
      if (!given) {
        if (wave == 0 && G.tile > 0) vp[0] = A.halo_in[2 * (G.gt - 1) + 1];
        if (wave == W - 1 && G.tile + 1 < G.ntile) vp[M + 1] = A.halo_in[2 * (G.gt + 1)];
      }
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t r = r0 + j;
      const bool ok = r < n;
      const double vm = fma(xv[j + 1], A.E_mat, A.vscale * vv[j + 1]);
      Ar[j] = mk(1.0, ok ? tau * (idx2 + vm) : 0.0);
      Br[j] = mk(0.0, (ok && r > 0) ? -kap : 0.0);
      Cr[j] = mk(0.0, (ok && r < n - 1) ? -kap : 0.0);
      if (given) {
        Dr[j] = vp[j + 1];
      } else {
        const double w = tau * (idx2 + fma(xv[j + 1], A.E_rhs, A.vscale * vv[j + 1]));
        const cd p = vp[j + 1];
        const cd s = cadd(vp[j], vp[j + 2]);
        Dr[j] = csel(ok, mk(fma(w, p.y, fma(-kap, s.y, p.x)), fma(-w, p.x, fma(kap, s.x, p.y))), zero);
      }
    }
    bK = mk(0.0, (r0 + M < n) ? -kap : 0.0);
    fst = vp[1];
    lst = vp[M];
  }
  if constexpr (PH == PH_REDUCE && halo_src(SRC)) {
    if (A.halo_out && live) {
      if (wave == 0) A.halo_out[2 * G.gt] = fst;
      if (wave == W - 1) A.halo_out[2 * G.gt + 1] = lst;
    }
  }
  Blk blk;
  if constexpr (RDR) {
    double ay[M];
#pragma unroll
    for (int j = 0; j < M; ++j) ay[j] = Ar[j].y;
    reduce_block_rd<M>(ay, CnEdges<false>{r0, n, kap}, Dr, bK.y, blk);
  } else {
    reduce_block<M, SRC == SRC_CN || SRC == SRC_LCOUP>(Ar, Br, Cr, Dr, bK, blk);
  }
  sm.blk[wave][lane] = blk;
  __syncthreads();
  if (wave == 0) {
    Blk acc = sm.blk[0][lane];
    for (int w = 1; w < W; ++w) {
      const Blk o = sm.blk[w][lane];
      Node t;
      merge_into(acc, o, t);
      *reinterpret_cast<Node*>(&sm.blk[w][lane]) = t;
    }
    cd pJ = zero, pM = zero;
    if constexpr (PH == PH_REDUCE) {
      if (live) {
        A.oU[3 * G.gt] = acc.UA;
        A.oU[3 * G.gt + 1] = acc.UC;
        A.oU[3 * G.gt + 2] = acc.UD;
        A.oD[3 * G.gt] = acc.DB;
        A.oD[3 * G.gt + 1] = acc.DA;
        A.oD[3 * G.gt + 2] = acc.DD;
      }
    } else {
      if constexpr (PH == PH_SINGLE) {
        cd ia0 = crecip(acc.UA);
        cd r = cneg(cmul(acc.DB, ia0));
        cd aT = cfma(r, acc.UC, cadd(mk(1.0, 0.0), acc.DA));
        cd dT = cfma(r, acc.UD, acc.DD);
        pM = cmul(dT, crecip(aT));
        pJ = cmul(cfms(acc.UC, pM, acc.UD), ia0);
      } else {
        pJ = A.psi_if[G.gt];
        const cd nxt = A.psi_if[(G.tile + 1 < G.ntile) ? G.gt + 1 : G.gt];
        pM = csel(G.tile + 1 < G.ntile, nxt, zero);
      }
      sm.jpsi[0][lane] = pJ;
      sm.jpsi[W][lane] = pM;
      cd right = pM;
      for (int w = W - 1; w >= 1; --w) {
        const Node t = *reinterpret_cast<const Node*>(&sm.blk[w][lane]);
        right = cfms(t.C, right, cfms(t.B, pJ, t.dl));
        sm.jpsi[w][lane] = right;
      }
    }
  }
  if constexpr (PH != PH_REDUCE) {
    __syncthreads();
    const cd pJ = sm.jpsi[wave][lane];
    const cd pK = sm.jpsi[wave + 1][lane];
    cd xo[M];
    ss_block<M>(Br, Cr, Dr, pJ, pK, xo);
    bool bad = false;
    const bool acc = (SRC == SRC_CN) && A.acc_pa != nullptr;
    double part = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int64_t r = r0 + j;
      if (live && r < n) {
        cd old = czero();
        if (acc && A.acc_half) old = col_at(A.x + c0, ob16, r, G.es);
        col_at(A.x + c0, ob16, r, G.es) = xo[j];
        bad |= !cfinite(xo[j]);
        if (acc) {
          const cd s = cadd(col_at(A.acc_pa + c0, ob16, r, G.es), col_at(A.acc_pb + c0, ob16, r, G.es));
          const cd lam =
              csel(A.acc_half != 0, mk(0.5 * (xo[j].x + old.x), 0.5 * (xo[j].y + old.y)), xo[j]);
          const double q = A.acc_tau * (lam.x * s.y - lam.y * s.x);
          if (A.acc_dV) col_at(A.acc_dV + c0, ob8, r, G.es) += A.vscale * q;
          if (A.xg) part = fma(col_at(A.xg + c0, ob8, r, G.es), q, part);
        }
      }
    }
    if (__any(bad) && lane == 0) atomicOr(A.status, 1);
    if (acc && A.acc_part) {
      sm.wpart[wave][lane] = part;
      __syncthreads();
      if (wave == 0 && live) {
        double t = 0.0;
        for (int w = 0; w < W; ++w) t += sm.wpart[w][lane];
        A.acc_part[G.gt] = t;
      }
    }
  }
}

// Reduced system on the joint lines of a system's tiles (K <= 64 rows, from the two slot
// arrays), solved by wavefront 0: lane k holds row k as a block without interior rows; the
// binary nesting reduces it to the RS stage on rows 0 and 64 (virtual) and SS gives psi at
// every tile joint.
__device__ __forceinline__ void interface_solve_wave(const cd* sU, const cd* sD, cd* spsi, int K,
                                                     int lane, Node* nodes) {
  const bool ok = lane < K;
  const int k = ok ? lane : 0;
  const cd zero = czero();
  cd a = sU[3 * k], c = sU[3 * k + 1], d = sU[3 * k + 2];
  const int kp = k > 0 ? k - 1 : 0;
  const cd da = sD[3 * kp + 1], dd = sD[3 * kp + 2];
  a = csel(k > 0, cadd(a, da), a);
  d = csel(k > 0, cadd(d, dd), d);
  const cd bn = sD[3 * k];  // sub-diagonal of row k+1
  Blk b;
  b.UA = csel(ok, a, mk(1.0, 0.0));
  b.UC = csel(lane < K - 1, c, zero);
  b.UD = csel(ok, d, zero);
  b.DB = csel(lane < K - 1, bn, zero);
  b.DA = zero;
  b.DD = zero;
  tree_up<6>(b, nodes, lane);
  cd pJ = zero, pM = zero;
  if (lane == 0) {
    cd ia0 = crecip(b.UA);
    cd r = cneg(cmul(b.DB, ia0));
    cd aT = cfma(r, b.UC, cadd(mk(1.0, 0.0), b.DA));
    cd dT = cfma(r, b.UD, b.DD);
    pM = cmul(dT, crecip(aT));
    pJ = cmul(cfms(b.UC, pM, b.UD), ia0);
  }
  tree_down<6>(pJ, pM, nodes, lane);
  if (ok) spsi[lane] = pJ;
}

constexpr int kMaxSysTiles = 64;

// Persistent launch over an uneven batch: every workgroup takes whole systems from a device
// queue (longest first, the host's order).  A system of at most one tile is solved in one
// pass; a longer one is streamed tile by tile inside the workgroup: reduce every tile (slots
// and edge states kept in LDS), solve the reduced system on the tile joints, then re-read each
// tile and substitute.  The last workgroup to leave resets the queue for the next launch.
template <int M, int W, int SRC>
__global__ __launch_bounds__(64 * W) void k_system(KArgs A) {
  constexpr int64_t T = 64 * W * M;
  __shared__ TileSmem<M, W> sm;
  __shared__ cd sU[3 * kMaxSysTiles], sD[3 * kMaxSysTiles], spsi[kMaxSysTiles],
      shalo[2 * kMaxSysTiles];
  __shared__ int item_s;
  KArgs B = A;
  B.oU = sU;
  B.oD = sD;
  B.psi_if = spsi;
  B.halo_out = shalo;
  B.halo_in = shalo;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(A.queue, 1);
    __syncthreads();
    const int item = item_s;
    __syncthreads();
    if (item >= A.nitems) break;
    Geo G;
    G.sys = A.wg_sys[item];
    G.base = A.offs[G.sys];
    G.cbase = G.base;
    G.n = A.offs[G.sys + 1] - G.base;
    G.es = 1;
    const int64_t K = (G.n + T - 1) / T;
    if (K <= 1) {
      G.tile = 0;
      G.gt = 0;
      G.ntile = 1;
      tile_run<M, W, SRC, PH_SINGLE>(A, G, sm);
    } else {
      G.ntile = K;
      for (int64_t t = 0; t < K; ++t) {
        G.tile = t;
        G.gt = t;
        tile_run<M, W, SRC, PH_REDUCE>(B, G, sm);
      }
      __syncthreads();
      if (wave == 0) interface_solve_wave(sU, sD, spsi, (int)K, lane, sm.xnode);
      __syncthreads();
      for (int64_t t = 0; t < K; ++t) {
        G.tile = t;
        G.gt = t;
        tile_run<M, W, SRC, PH_SUBST>(B, G, sm);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(A.queue + 1, 1) == (int)gridDim.x - 1) {
      atomicExch(A.queue, 0);
      atomicExch(A.queue + 1, 0);
    }
  }
}

// ------------------------------------------------------------------------ auxiliary kernels
struct AuxArgs {
  int64_t n, batch, es, bs;
  const int64_t* offs;
  int64_t total;  // total rows (uneven) or n*batch
  const double* V;
  const double* xg;
  double vscale, E, dx, dt;
  const double* dxs;
  const double* W;  // absorbing potential (the potential is V - i wscale W), or null
  double wscale;
  const cd* psi;
  cd *a, *b, *c, *d;
  // adjoint accumulation
  const cd* lam;
  const cd* psi_n;
  const cd* psi_np1;
  double* dV;
  double* dE_part;
  // solve gradients
  const cd* xsol;
  cd *ga, *gb, *gc;
  // partial-wave step: first partial wave of the batch
  int64_t l0;
};

}  // namespace nsd
