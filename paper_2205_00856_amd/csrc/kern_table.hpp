// Kernel tables of the library: the tile configurations and the host-side entry addresses of
// every kernel instantiation.  Each kern_*.hip unit instantiates one group of kernels and
// fills its part of the table, so the units compile in parallel and the host runtime
// (cntri.hip) never instantiates a kernel template itself.
#pragma once
#include <stdint.h>

#include <utility>

namespace nsk {

struct Cfg {
  int M, W;
  constexpr int64_t T() const { return 64LL * W * M; }
};
// Row tiles (k_tile, k_system): (rows per lane, wavefronts per workgroup); T = 64 W M rows.
// {1, 1} (a 64-row partition, every lane's block one joint row) is built for the explicit
// sources and the reduced systems only.
constexpr Cfg kCfgs[] = {{2, 1}, {4, 1}, {4, 2}, {4, 4}, {4, 8}, {4, 16}, {8, 1}, {8, 2},
                         {8, 4}, {8, 8}, {2, 2}, {2, 4}, {16, 4}, {16, 2}, {1, 1}};
constexpr int kNumCfg = sizeof(kCfgs) / sizeof(kCfgs[0]);
// Column tiles of interleaved batches (k_cols): T = W M rows of 64 neighbouring systems.
constexpr Cfg kColCfgs[] = {{4, 8}, {8, 4}, {8, 8}, {4, 16}, {16, 4}, {8, 16}};
constexpr int kNumColCfg = sizeof(kColCfgs) / sizeof(kColCfgs[0]);

// Resident propagations (k_resident): 8 rows per lane, tiles of 512, 1024 and 2048 rows.
constexpr Cfg kResCfgs[] = {{8, 1}, {8, 2}, {8, 4}};
constexpr int kNumResCfg = sizeof(kResCfgs) / sizeof(kResCfgs[0]);

constexpr int kNumSrc = 6;  // nsd::Src
constexpr int kNumPh = 4;   // nsd::Phase

enum AuxKernel : int {
  AUX_ASSEMBLE = 0,
  AUX_RHS,
  AUX_SOLVE_GRADS,
  AUX_ADJ_ACCUM,
  AUX_SUM_PARTIALS,
  AUX_RS_SERIAL,
  AUX_RADIAL_VEFF,
  AUX_RADIAL_COUPLING,
  kNumAux
};

struct Tables {
  const void* tile[kNumCfg][kNumSrc][kNumPh];
  const void* pers[kNumCfg][kNumSrc];
  const void* cols[kNumColCfg][kNumSrc][3];
  const void* mrhs[kNumCfg][3];  // one matrix, several right-hand sides (explicit source)
  const void* aux[kNumAux];
  const void* res[kNumResCfg][2];  // resident propagation of one system: [SRC_CN, SRC_CNW]
  // explicit solve with first-level partitions of C = 2 or 4 chunks of 4096 rows (8192 and
  // 16384 rows, k_tile_chunk): [C == 4][0: PH_REDUCE, 1: PH_SUBST]
  const void* chunk[2][2];
};

// The one table of the library (cntri.hip), filled once by the registration functions below.
Tables& tables();

void reg_tile_expl(Tables& t);
void reg_tile_ct(Tables& t);
void reg_tile_cn_lo(Tables& t);
void reg_tile_cn_hi(Tables& t);
void reg_tile_cnw(Tables& t);
void reg_tile_slots(Tables& t);
void reg_cols(Tables& t);
void reg_pers(Tables& t);
void reg_mrhs(Tables& t);
void reg_aux(Tables& t);
void reg_resident(Tables& t);

template <int M, int W>
constexpr int cfg_index() {
  for (int i = 0; i < kNumCfg; ++i)
    if (kCfgs[i].M == M && kCfgs[i].W == W) return i;
  return -1;
}
template <int M, int W>
constexpr int col_cfg_index() {
  for (int i = 0; i < kNumColCfg; ++i)
    if (kColCfgs[i].M == M && kColCfgs[i].W == W) return i;
  return -1;
}

}  // namespace nsk
