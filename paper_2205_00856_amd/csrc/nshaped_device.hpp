// Device building blocks of the N-shaped partition solver for gfx950 (FP64 complex).
//
// Method: arXiv 2205.00856, Sec. 4 and Table 1.  One workgroup owns a "tile" of
// T = 64 * W * M consecutive rows of one system and applies the method nested over three
// granularities (Sec. 4.1.6, Eq. (6)):
//   level 1  each lane owns a block of M rows: its top joint line J plus M-1 interior rows.
//            RD+JD then RU+JU run on the block in registers (Table 1, in the order of
//            Sec. 5.2.1).
//   level 2+ the joint lines of neighbouring blocks form a reduced tridiagonal system; it is
//            reduced again with blocks that contain exactly one interior joint line, for
//            which RD/RU are empty and JU/JD are one elimination each.  Inside a wavefront
//            the pairs exchange data with cross-lane moves (6 levels), across the W
//            wavefronts of the workgroup through LDS (log2 W levels).
//   top      either the RS stage on the tile's two joint lines (whole system in one tile),
//            or the tile's two joint-line "slots" are written out so that the reduced system
//            over all tiles is solved by the same method one level up.
// SS runs the other way: from the tile's joint lines down the tree to every row.
//
// Every reduced row is scaled by its pivot as soon as the pivot is known (the 1/a_i
// precompute of Sec. 5.2.2 applied in place), so a reduced interior row is stored as
//     psi_i + beta_i psi_J + gamma_i psi_K = delta_i
// and SS is psi_i = delta_i - beta_i psi_J - gamma_i psi_K.  Table 1's updates become
//   RD (row i-1 scaled):  r = -b_i;       a_i += r gamma_{i-1}; b_i = r beta_{i-1}; d_i += r delta_{i-1}
//   RU (row i+1 final):   r = -gamma_i;   beta_i += r beta_{i+1}; gamma_i = r gamma_{i+1}; delta_i += r delta_{i+1}
// which are the printed operations applied to the row-scaled system.
//
// Block state ("two slots", Sec. 4.1.3): a reduced block [J, K] contributes
//   to row J (U slot, own row folded in):  UA psi_J + UC psi_K = UD
//   to row K (D slot):                     DB psi_J + DA psi_K = DD
// and the reader adds the slots in a fixed order, so no floating-point atomics are used.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsd {

typedef double2 cd;

__device__ __forceinline__ cd mk(double r, double i) {
  cd z;
  z.x = r;
  z.y = i;
  return z;
}
__device__ __forceinline__ cd czero() { return mk(0.0, 0.0); }
__device__ __forceinline__ cd cadd(cd a, cd b) { return mk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cd csub(cd a, cd b) { return mk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cd cneg(cd a) { return mk(-a.x, -a.y); }
__device__ __forceinline__ cd cconj(cd a) { return mk(a.x, -a.y); }
__device__ __forceinline__ cd cmul(cd a, cd b) {
  return mk(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// acc + a * b
__device__ __forceinline__ cd cfma(cd a, cd b, cd acc) {
  return mk(fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y)));
}
// acc - a * b
__device__ __forceinline__ cd cfms(cd a, cd b, cd acc) {
  return mk(fma(-a.x, b.x, fma(a.y, b.y, acc.x)), fma(-a.x, b.y, fma(-a.y, b.x, acc.y)));
}
__device__ __forceinline__ cd csel(bool p, cd a, cd b) { return mk(p ? a.x : b.x, p ? a.y : b.y); }

// 1/v from the hardware estimate refined by two Newton-Raphson steps
// x <- x + x (1 - v x)  (Newton's iteration for the reciprocal; the error squares per step).
__device__ __forceinline__ double rcp_nr(double v) {
  double r = __builtin_amdgcn_rcp(v);
  double e = fma(-v, r, 1.0);
  r = fma(r, e, r);
  e = fma(-v, r, 1.0);
  r = fma(r, e, r);
  return r;
}
// 1/a = conj(a) / |a|^2  (valid while |a|^2 is a normal double)
__device__ __forceinline__ cd crecip(cd a) {
  double s = rcp_nr(fma(a.x, a.x, a.y * a.y));
  return mk(a.x * s, -a.y * s);
}
__device__ __forceinline__ bool cfinite(cd a) { return isfinite(a.x) && isfinite(a.y); }

struct Blk {
  cd UA, UC, UD;  // U slot: contribution to (and own data of) the top joint row
  cd DB, DA, DD;  // D slot: contribution to the bottom joint row
};
// one eliminated joint line K between J and M, scaled:  psi_K = dl - B psi_J - C psi_M
struct Node {
  cd B, C, dl;
};

// ---------------------------------------------------------------- level 1: one lane's block
// (i b) z for a pure imaginary i b
__device__ __forceinline__ cd cimul(double b, cd z) { return mk(-b * z.y, b * z.x); }

// Input rows J .. J+M-1 (local 0 .. M-1) as (a, b, c, d) in (A, Bt, Ct, D); bK is the
// sub-diagonal of the next joint line K = J+M.  On return rows 1..M-1 hold the scaled reduced
// rows (beta in Bt, gamma in Ct, delta in D) for SS; A is consumed.  With IMAG the input
// off-diagonals (b, c, bK) are pure imaginary (only their imaginary parts are read), as in
// every Crank-Nicolson matrix with a real potential.
template <int M, bool IMAG = false>
__device__ __forceinline__ void reduce_block(cd (&A)[M], cd (&Bt)[M], cd (&Ct)[M], cd (&D)[M],
                                             cd bK, Blk& o) {
  auto bmul = [](cd b, cd z) { return IMAG ? cimul(b.y, z) : cmul(b, z); };
  if constexpr (M == 1) {
    // a block without interior rows: its two joint lines are coupled directly
    o.UA = A[0];
    o.UC = Ct[0];
    o.UD = D[0];
    o.DB = bK;
    o.DA = czero();
    o.DD = czero();
  } else {
    // row J+1 keeps its b (coefficient of psi_J); scale it by its pivot
    {
      cd ia = crecip(A[1]);
      Bt[1] = bmul(Bt[1], ia);
      Ct[1] = bmul(Ct[1], ia);
      D[1] = cmul(D[1], ia);
    }
    // RD: i = J+2 .. K-1 with row i-1 scaled: r = -b_i
#pragma unroll
    for (int i = 2; i < M; ++i) {
      cd a = csub(A[i], bmul(Bt[i], Ct[i - 1]));  // a_i - b_i gamma_{i-1}
      cd d = csub(D[i], bmul(Bt[i], D[i - 1]));   // d_i - b_i delta_{i-1}
      cd b = cneg(bmul(Bt[i], Bt[i - 1]));        // -b_i beta_{i-1}
      cd ia = crecip(a);
      Bt[i] = cmul(b, ia);
      Ct[i] = bmul(Ct[i], ia);
      D[i] = cmul(d, ia);
    }
    // JD at K: r = -b_K (row K-1 scaled)
    o.DB = cneg(bmul(bK, Bt[M - 1]));
    o.DA = cneg(bmul(bK, Ct[M - 1]));
    o.DD = cneg(bmul(bK, D[M - 1]));
    // RU: i = K-2 .. J+1 with row i+1 final: r = -gamma_i
#pragma unroll
    for (int i = M - 2; i >= 1; --i) {
      cd g = Ct[i];
      Bt[i] = cfms(g, Bt[i + 1], Bt[i]);
      D[i] = cfms(g, D[i + 1], D[i]);
      Ct[i] = cneg(cmul(g, Ct[i + 1]));
    }
    // JU at J: r = -c_J (row J+1 final)
    o.UA = csub(A[0], bmul(Ct[0], Bt[1]));
    o.UD = csub(D[0], bmul(Ct[0], D[1]));
    o.UC = cneg(bmul(Ct[0], Ct[1]));
  }
}

// Off-diagonals of a Crank-Nicolson block: rows J .. J+M-1 of a system of n rows, each coupled
// to its neighbours by -i kappa, except across the system ends and on padding rows past n.
// IN: the caller knows every row of the block and both neighbours lie inside the system.
template <bool IN>
struct CnEdges {
  int64_t J, n;
  double kap;
  // imaginary parts of the sub- and super-diagonal of local row i
  __device__ __forceinline__ double b(int i) const {
    const int64_t r = J + i;
    return (IN || (r < n && r > 0)) ? -kap : 0.0;
  }
  __device__ __forceinline__ double c(int i) const {
    const int64_t r = J + i;
    return (IN || r < n - 1) ? -kap : 0.0;
  }
};

// Level 1 with substitution along the RD rows (Crank-Nicolson blocks, M >= 2).  ay holds the
// imaginary parts of the diagonal (real parts 1), e the off-diagonals, bK the imaginary part of
// the sub-diagonal of the next joint line.  RD and JD are reduce_block's operations; rows
// 1..M-1 keep their RD form
//     psi_i + beta_i psi_J + gamma_i psi_{i+1} = delta_i
// with only delta_i retained (in D): beta_i and gamma_i depend on the matrix alone and are
// recomputed by ss_block_rd, so a lane carries one complex value per row across the nesting
// levels instead of three.  RU only has to deliver the final row J+1 for JU; unrolled, that row
// is the forward sum  psi_{J+1} = sum_k P_k (delta_k - beta_k psi_J) + P_M psi_K  with P_1 = 1,
// P_{k+1} = -gamma_k P_k, accumulated here during RD, so no RD row is held for a backward pass.
// CR: the diagonal's real parts are ar instead of 1 (a Crank-Nicolson matrix with an absorbing
// potential: 1 + tau W); the off-diagonals stay those of e.
template <int M, bool CR, typename E>
__device__ __forceinline__ void reduce_block_rd_g(const double (&ar)[M], const double (&ay)[M],
                                                  const E& e, cd (&D)[M], double bK, Blk& o) {
  static_assert(M >= 2, "blocks with interior rows");
  auto dg = [&](int i) { return mk(CR ? ar[i] : 1.0, ay[i]); };
  cd beta, gam;
  {
    const cd ia = crecip(dg(1));
    beta = cimul(e.b(1), ia);
    gam = cimul(e.c(1), ia);
    D[1] = cmul(D[1], ia);
  }
  cd fb = beta, fd = D[1], P = cneg(gam);
#pragma unroll
  for (int i = 2; i < M; ++i) {
    const double bi = e.b(i);
    const cd a = csub(dg(i), cimul(bi, gam));
    const cd d = csub(D[i], cimul(bi, D[i - 1]));
    const cd b = cneg(cimul(bi, beta));
    const cd ia = crecip(a);
    beta = cmul(b, ia);
    gam = cimul(e.c(i), ia);
    D[i] = cmul(d, ia);
    fb = cfma(P, beta, fb);
    fd = cfma(P, D[i], fd);
    P = cneg(cmul(P, gam));
  }
  // JD at K (row K-1 scaled)
  o.DB = cneg(cimul(bK, beta));
  o.DA = cneg(cimul(bK, gam));
  o.DD = cneg(cimul(bK, D[M - 1]));
  // JU at J with row J+1 final: beta = fb, gamma = -P, delta = fd
  const double c0 = e.c(0);
  o.UA = csub(dg(0), cimul(c0, fb));
  o.UD = csub(D[0], cimul(c0, fd));
  o.UC = cimul(c0, P);
}
template <int M, typename E>
__device__ __forceinline__ void reduce_block_rd(const double (&ay)[M], const E& e,
                                                cd (&D)[M], double bK, Blk& o) {
  reduce_block_rd_g<M, false>(ay, ay, e, D, bK, o);
}

// SS along the RD rows of reduce_block_rd(_g): with psi_J and psi_K = psi_{J+M} known,
//   psi_i = delta_i - beta_i psi_J - gamma_i psi_{i+1},  i = M-1 down to 1,
// where beta_i and gamma_i are recomputed from ay and e with reduce_block_rd's operations.
template <int M, bool CR, typename E>
__device__ __forceinline__ void ss_block_rd_g(const double (&ar)[M], const double (&ay)[M],
                                              const E& e, const cd (&D)[M], cd pJ, cd pK,
                                              cd (&x)[M]) {
  auto dg = [&](int i) { return mk(CR ? ar[i] : 1.0, ay[i]); };
  cd gam[M], dp[M];
  cd beta;
  {
    const cd ia = crecip(dg(1));
    beta = cimul(e.b(1), ia);
    gam[1] = cimul(e.c(1), ia);
    dp[1] = cfms(beta, pJ, D[1]);
  }
#pragma unroll
  for (int i = 2; i < M; ++i) {
    const double bi = e.b(i);
    const cd a = csub(dg(i), cimul(bi, gam[i - 1]));
    const cd ia = crecip(a);
    beta = cmul(cneg(cimul(bi, beta)), ia);
    gam[i] = cimul(e.c(i), ia);
    dp[i] = cfms(beta, pJ, D[i]);
  }
  x[0] = pJ;
  cd nx = pK;
#pragma unroll
  for (int i = M - 1; i >= 1; --i) {
    nx = cfms(gam[i], nx, dp[i]);
    x[i] = nx;
  }
}
template <int M, typename E>
__device__ __forceinline__ void ss_block_rd(const double (&ay)[M], const E& e,
                                            const cd (&D)[M], cd pJ, cd pK, cd (&x)[M]) {
  ss_block_rd_g<M, false>(ay, ay, e, D, pJ, pK, x);
}

// SS on the lane's block: psi_i = delta_i - beta_i psi_J - gamma_i psi_K.
template <int M>
__device__ __forceinline__ void ss_block(const cd (&Bt)[M], const cd (&Ct)[M], const cd (&D)[M],
                                         cd pJ, cd pK, cd (&x)[M]) {
  x[0] = pJ;
#pragma unroll
  for (int i = 1; i < M; ++i) x[i] = cfms(Ct[i], pK, cfms(Bt[i], pJ, D[i]));
}

// ------------------------------------------------------------------ cross-lane xor moves
// lane i receives the value of lane i ^ m (m a power of two below 64)
template <int m>
__device__ __forceinline__ int xmove(int v) {
  if constexpr (m == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (m == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (m == 4) {
    return __builtin_amdgcn_ds_swizzle(v, 0x101F);  // bitmask mode, xor 0x04 within 32 lanes
  } else if constexpr (m == 8) {
    return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (m == 16) {
    return __builtin_amdgcn_ds_swizzle(v, 0x401F);  // bitmask mode, xor 0x10 within 32 lanes
  } else {
    return __shfl_xor(v, m, 64);
  }
}
template <int m>
__device__ __forceinline__ double xmove(double v) {
  int2 t = __builtin_bit_cast(int2, v);
  t.x = xmove<m>(t.x);
  t.y = xmove<m>(t.y);
  return __builtin_bit_cast(double, t);
}
template <int m>
__device__ __forceinline__ cd xmove(cd v) {
  return mk(xmove<m>(v.x), xmove<m>(v.y));
}

// ------------------------------------------------------------- level 2+: pairs of blocks
// L = [J, K], R = [K, M]: eliminate joint line K (the single interior row of [J, M]).
//   row K: DB_L psi_J + (DA_L + UA_R) psi_K + UC_R psi_M = DD_L + UD_R, scaled by its pivot:
//          psi_K + B psi_J + C psi_M = dl
//   JU at J: r = -UC_L: UA += r B; UC = r C; UD += r dl
//   JD at M: r = -DB_R: DB = r B;  DA += r C; DD += r dl
// At level s the lanes with the low s bits clear take part: lane x (bit s clear) holds L and
// lane x + 2^s holds R.  The lane of L receives R, keeps the merged block and stores the
// scaled row K in LDS slot x + 2^s (read back by the same lane in SS).  The other lanes
// compute the same formulas on data that is no longer needed.
// b = [J, K] absorbs o = [K, M]: b becomes [J, M]; t is the scaled row K.
__device__ __forceinline__ void merge_into(Blk& b, const Blk& o, Node& t) {
  const cd ia = crecip(cadd(b.DA, o.UA));
  t.B = cmul(b.DB, ia);
  t.C = cmul(o.UC, ia);
  t.dl = cmul(cadd(b.DD, o.UD), ia);
  const cd rU = b.UC;
  const cd rD = o.DB;
  b.UA = cfms(rU, t.B, b.UA);
  b.UD = cfms(rU, t.dl, b.UD);
  b.UC = cneg(cmul(rU, t.C));
  b.DB = cneg(cmul(rD, t.B));
  b.DA = cfms(rD, t.C, o.DA);
  b.DD = cfms(rD, t.dl, o.DD);
}

template <int m>
__device__ __forceinline__ void tree_level_up(Blk& b, Node* nodes, int lane) {
  Blk o;
  o.UA = xmove<m>(b.UA);
  o.UC = xmove<m>(b.UC);
  o.UD = xmove<m>(b.UD);
  o.DB = xmove<m>(b.DB);
  o.DA = xmove<m>(b.DA);
  o.DD = xmove<m>(b.DD);
  Node t;
  merge_into(b, o, t);
  if ((lane & (2 * m - 1)) == 0) nodes[lane + m] = t;
}

// Binary nesting over 2^LEVELS consecutive lanes: afterwards the lane with the low LEVELS bits
// clear holds the merged block; the nodes of the eliminated joint lines are in `nodes`.
template <int LEVELS>
__device__ __forceinline__ void tree_up(Blk& b, Node* nodes, int lane) {
  if constexpr (LEVELS > 0) tree_level_up<1>(b, nodes, lane);
  if constexpr (LEVELS > 1) tree_level_up<2>(b, nodes, lane);
  if constexpr (LEVELS > 2) tree_level_up<4>(b, nodes, lane);
  if constexpr (LEVELS > 3) tree_level_up<8>(b, nodes, lane);
  if constexpr (LEVELS > 4) tree_level_up<16>(b, nodes, lane);
  if constexpr (LEVELS > 5) tree_level_up<32>(b, nodes, lane);
}

// SS at level s: the lane of L knows (psi_J, psi_M), computes psi_K and hands (psi_K, psi_M)
// to the lane of R.
template <int m>
__device__ __forceinline__ void tree_level_down(cd& pJ, cd& pM, const Node* nodes, int lane) {
  const Node t = nodes[(lane + m) & 63];
  const cd pK = cfms(t.C, pM, cfms(t.B, pJ, t.dl));
  const cd oK = xmove<m>(pK);
  const cd oM = xmove<m>(pM);
  const int low = lane & (2 * m - 1);
  if (low == m) {
    pJ = oK;
    pM = oM;
  }
  if (low == 0) pM = pK;
}

// SS down the binary nesting: on entry the group's first lane holds (psi_J, psi_M) of the whole
// span; on exit every lane holds psi at its own joint line (pJ) and at the next one (pM).
template <int LEVELS>
__device__ __forceinline__ void tree_down(cd& pJ, cd& pM, const Node* nodes, int lane) {
  if constexpr (LEVELS > 5) tree_level_down<32>(pJ, pM, nodes, lane);
  if constexpr (LEVELS > 4) tree_level_down<16>(pJ, pM, nodes, lane);
  if constexpr (LEVELS > 3) tree_level_down<8>(pJ, pM, nodes, lane);
  if constexpr (LEVELS > 2) tree_level_down<4>(pJ, pM, nodes, lane);
  if constexpr (LEVELS > 1) tree_level_down<2>(pJ, pM, nodes, lane);
  if constexpr (LEVELS > 0) tree_level_down<1>(pJ, pM, nodes, lane);
}

// ------------------------------------------- several right-hand sides of one matrix (factored)
// The multipliers of RD, JD, RU and JU (the r factors of Table 1) and the pivots depend on the
// matrix alone; only the updates of d involve the right-hand side (Sec. 5.2.4 keeps the r
// factors for this reason).  The functions below split reduce_block and merge_into into a
// matrix part, run once per tile, and a right-hand-side part, run for each right-hand side.
// Together they perform the very operations of the unsplit functions on the same operands in
// the same order, so each right-hand side gets the same bits as a solve of its own.

// The factors of one lane's block (general complex rows).
template <int M>
struct BlkFac {
  cd ia[M];         // ia[i] (i >= 1): reciprocal of the pivot of row J+i
  cd b[M];          // b[i] (i >= 2): the RD multiplier of delta_{i-1} in row J+i
  cd g[M];          // g[i] (1 <= i <= M-2): the RU multiplier gamma_i of delta_{i+1}
  cd c0, bK;        // the JU multiplier c_J and the JD multiplier b_K
  cd Bt[M], Ct[M];  // the reduced rows (beta, gamma) that SS applies to psi_J and psi_K
};

// Matrix part of reduce_block (no IMAG): o receives UA, UC, DB, DA; F the factors.
template <int M>
__device__ __forceinline__ void reduce_block_fac(const cd (&A)[M], const cd (&B)[M],
                                                 const cd (&C)[M], cd bK, BlkFac<M>& F,
                                                 Blk& o) {
  F.c0 = C[0];
  F.bK = bK;
  if constexpr (M == 1) {
    o.UA = A[0];
    o.UC = C[0];
    o.DB = bK;
    o.DA = czero();
  } else {
    cd Bt[M], Ct[M];
    {
      const cd ia = crecip(A[1]);
      F.ia[1] = ia;
      Bt[1] = cmul(B[1], ia);
      Ct[1] = cmul(C[1], ia);
    }
#pragma unroll
    for (int i = 2; i < M; ++i) {
      const cd a = csub(A[i], cmul(B[i], Ct[i - 1]));
      const cd b = cneg(cmul(B[i], Bt[i - 1]));
      const cd ia = crecip(a);
      F.ia[i] = ia;
      F.b[i] = B[i];
      Bt[i] = cmul(b, ia);
      Ct[i] = cmul(C[i], ia);
    }
    o.DB = cneg(cmul(bK, Bt[M - 1]));
    o.DA = cneg(cmul(bK, Ct[M - 1]));
#pragma unroll
    for (int i = M - 2; i >= 1; --i) {
      const cd g = Ct[i];
      F.g[i] = g;
      Bt[i] = cfms(g, Bt[i + 1], Bt[i]);
      Ct[i] = cneg(cmul(g, Ct[i + 1]));
    }
    o.UA = csub(A[0], cmul(C[0], Bt[1]));
    o.UC = cneg(cmul(C[0], Ct[1]));
#pragma unroll
    for (int i = 1; i < M; ++i) {
      F.Bt[i] = Bt[i];
      F.Ct[i] = Ct[i];
    }
  }
}

// Right-hand-side part of reduce_block: D becomes the deltas that SS reads; UD, DD the block's
// right-hand sides at its two joint lines.
template <int M>
__device__ __forceinline__ void reduce_block_rhs(const BlkFac<M>& F, cd (&D)[M], cd& UD,
                                                 cd& DD) {
  if constexpr (M == 1) {
    UD = D[0];
    DD = czero();
  } else {
    D[1] = cmul(D[1], F.ia[1]);
#pragma unroll
    for (int i = 2; i < M; ++i) {
      const cd d = csub(D[i], cmul(F.b[i], D[i - 1]));
      D[i] = cmul(d, F.ia[i]);
    }
    DD = cneg(cmul(F.bK, D[M - 1]));
#pragma unroll
    for (int i = M - 2; i >= 1; --i) D[i] = cfms(F.g[i], D[i + 1], D[i]);
    UD = csub(D[0], cmul(F.c0, D[1]));
  }
}

// An eliminated joint line K of the nesting, matrix part: its scaled row (B, C) for SS, the
// reciprocal of its pivot and the JU / JD multipliers that fold its right-hand side into the
// merged block.
struct NodeFac {
  cd B, C, ia, rU, rD;
};

// Matrix part of merge_into (UA, UC, DB, DA of b and o).
__device__ __forceinline__ void merge_fac(Blk& b, const Blk& o, NodeFac& t) {
  const cd ia = crecip(cadd(b.DA, o.UA));
  t.B = cmul(b.DB, ia);
  t.C = cmul(o.UC, ia);
  t.ia = ia;
  t.rU = b.UC;
  t.rD = o.DB;
  b.UA = cfms(t.rU, t.B, b.UA);
  b.UC = cneg(cmul(t.rU, t.C));
  b.DB = cneg(cmul(t.rD, t.B));
  b.DA = cfms(t.rD, t.C, o.DA);
}

// Right-hand-side part of merge_into: (UD, DD) of [J, K] absorbs (oUD, oDD) of [K, M]; returns
// the scaled right-hand side dl of row K.
__device__ __forceinline__ cd merge_rhs(cd& UD, cd& DD, cd oUD, cd oDD, cd ia, cd rU, cd rD) {
  const cd dl = cmul(cadd(DD, oUD), ia);
  UD = cfms(rU, dl, UD);
  DD = cfms(rD, dl, oDD);
  return dl;
}

// The nesting levels of tree_up, matrix part: the lane of L keeps the factors of row K in
// f[lane + m] (the slot tree_up gives its node); the right-hand-side part reads them back in
// the same lane.
template <int m>
__device__ __forceinline__ void tree_level_up_fac(Blk& b, NodeFac* f, int lane) {
  Blk o;
  o.UA = xmove<m>(b.UA);
  o.UC = xmove<m>(b.UC);
  o.DB = xmove<m>(b.DB);
  o.DA = xmove<m>(b.DA);
  NodeFac t;
  merge_fac(b, o, t);
  if ((lane & (2 * m - 1)) == 0) f[lane + m] = t;
}

template <int LEVELS>
__device__ __forceinline__ void tree_up_fac(Blk& b, NodeFac* f, int lane) {
  if constexpr (LEVELS > 0) tree_level_up_fac<1>(b, f, lane);
  if constexpr (LEVELS > 1) tree_level_up_fac<2>(b, f, lane);
  if constexpr (LEVELS > 2) tree_level_up_fac<4>(b, f, lane);
  if constexpr (LEVELS > 3) tree_level_up_fac<8>(b, f, lane);
  if constexpr (LEVELS > 4) tree_level_up_fac<16>(b, f, lane);
  if constexpr (LEVELS > 5) tree_level_up_fac<32>(b, f, lane);
}

template <int m>
__device__ __forceinline__ void tree_level_up_rhs(cd& UD, cd& DD, const NodeFac* __restrict__ f,
                                                  cd* __restrict__ dl, int lane) {
  const NodeFac& t = f[(lane + m) & 63];
  const cd oUD = xmove<m>(UD);
  const cd oDD = xmove<m>(DD);
  const cd d = merge_rhs(UD, DD, oUD, oDD, t.ia, t.rU, t.rD);
  if ((lane & (2 * m - 1)) == 0) dl[lane + m] = d;
}

// Right-hand-side part of tree_up: the levels run on (UD, DD) alone with the factors of the
// matrix part; dl receives the scaled right-hand sides of the eliminated rows in the node slots.
template <int LEVELS>
__device__ __forceinline__ void tree_up_rhs(cd& UD, cd& DD, const NodeFac* __restrict__ f,
                                            cd* __restrict__ dl, int lane) {
  if constexpr (LEVELS > 0) tree_level_up_rhs<1>(UD, DD, f, dl, lane);
  if constexpr (LEVELS > 1) tree_level_up_rhs<2>(UD, DD, f, dl, lane);
  if constexpr (LEVELS > 2) tree_level_up_rhs<4>(UD, DD, f, dl, lane);
  if constexpr (LEVELS > 3) tree_level_up_rhs<8>(UD, DD, f, dl, lane);
  if constexpr (LEVELS > 4) tree_level_up_rhs<16>(UD, DD, f, dl, lane);
  if constexpr (LEVELS > 5) tree_level_up_rhs<32>(UD, DD, f, dl, lane);
}

// tree_level_down with the node split into its matrix part (f) and its right-hand side (dl).
template <int m>
__device__ __forceinline__ void tree_level_down_fac(cd& pJ, cd& pM, const NodeFac* f,
                                                    const cd* dl, int lane) {
  const int k = (lane + m) & 63;
  const cd pK = cfms(f[k].C, pM, cfms(f[k].B, pJ, dl[k]));
  const cd oK = xmove<m>(pK);
  const cd oM = xmove<m>(pM);
  const int low = lane & (2 * m - 1);
  if (low == m) {
    pJ = oK;
    pM = oM;
  }
  if (low == 0) pM = pK;
}

template <int LEVELS>
__device__ __forceinline__ void tree_down_fac(cd& pJ, cd& pM, const NodeFac* f, const cd* dl,
                                              int lane) {
  if constexpr (LEVELS > 5) tree_level_down_fac<32>(pJ, pM, f, dl, lane);
  if constexpr (LEVELS > 4) tree_level_down_fac<16>(pJ, pM, f, dl, lane);
  if constexpr (LEVELS > 3) tree_level_down_fac<8>(pJ, pM, f, dl, lane);
  if constexpr (LEVELS > 2) tree_level_down_fac<4>(pJ, pM, f, dl, lane);
  if constexpr (LEVELS > 1) tree_level_down_fac<2>(pJ, pM, f, dl, lane);
  if constexpr (LEVELS > 0) tree_level_down_fac<1>(pJ, pM, f, dl, lane);
}

// ------------------------------------------------------------------ LDS staging per wavefront
// A wavefront covers rows w0 .. w0+64M-1 plus one halo row on each side.  Global loads and
// stores are coalesced (lane l touches row w0 + 64k + l); the lane-to-block transposition goes
// through LDS, padded by one element per M rows so that lane strides of M+1 elements are free
// of bank conflicts.
template <int M>
struct Stage {
  static constexpr int QN = 64 * M + 2;  // staged rows: w0-1 .. w0+64M
  // padded length; at least 192 complex values, the 64 tree nodes the buffer holds in between
  static constexpr int QS = (QN + QN / M + 2) < 192 ? 192 : (QN + QN / M + 2);
  __device__ static __forceinline__ int addr(int q) { return q + q / M; }
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace nsd
