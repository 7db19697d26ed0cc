// Row-tile kernels (k_tile) of the Crank-Nicolson step with an absorbing potential (operator
// assembled in-kernel with T's diagonal 1 + tau W + i tau (...)): the configurations that the
// plans of such steps use (whole systems up to 4096 rows; tiles of 4 rows per lane for longer
// ones).
#include "kern_table.hpp"
#include "nshaped_kernels.hpp"

namespace nsk {
namespace {
// every phase (tiles of multi-tile systems and the fused pass of a sequence)
template <int M, int W>
void reg_all(Tables& t) {
  constexpr int I = cfg_index<M, W>();
  static_assert(I >= 0, "a configuration of the row-tile table");
  constexpr int S = nsd::SRC_CNW;
  t.tile[I][S][nsd::PH_SINGLE] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_SINGLE>;
  t.tile[I][S][nsd::PH_REDUCE] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_REDUCE>;
  t.tile[I][S][nsd::PH_SUBST] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_SUBST>;
  t.tile[I][S][nsd::PH_FUSE] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_FUSE>;
}
// whole systems in one tile only
template <int M, int W>
void reg_single(Tables& t) {
  constexpr int I = cfg_index<M, W>();
  static_assert(I >= 0, "a configuration of the row-tile table");
  t.tile[I][nsd::SRC_CNW][nsd::PH_SINGLE] =
      (const void*)&nsd::k_tile<M, W, nsd::SRC_CNW, nsd::PH_SINGLE>;
}
}  // namespace

void reg_tile_cnw(Tables& t) {
  reg_all<2, 1>(t);
  reg_all<4, 1>(t);
  reg_all<4, 2>(t);
  reg_all<4, 4>(t);
  reg_all<8, 4>(t);
  reg_single<8, 8>(t);
}

}  // namespace nsk
