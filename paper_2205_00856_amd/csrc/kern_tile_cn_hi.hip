// Row-tile kernels (k_tile) of the Crank-Nicolson step (operator assembled in-kernel): every tile configuration 7 and up.
#include "kern_table.hpp"
#include "nshaped_kernels.hpp"

namespace nsk {
namespace {
template <int I>
void reg_one(Tables& t) {
  constexpr int M = kCfgs[I].M, W = kCfgs[I].W;
  constexpr int S = nsd::SRC_CN;
  if constexpr (M >= 2) {  // the fused pass reduces in the RD form, which needs interior rows
    t.tile[I][S][nsd::PH_SINGLE] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_SINGLE>;
    t.tile[I][S][nsd::PH_REDUCE] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_REDUCE>;
    t.tile[I][S][nsd::PH_SUBST] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_SUBST>;
    t.tile[I][S][nsd::PH_FUSE] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_FUSE>;
  }
}
template <int... I>
void reg_range(Tables& t, std::integer_sequence<int, I...>) {
  (reg_one<I + 7>(t), ...);
}
}  // namespace

void reg_tile_cn_hi(Tables& t) { reg_range(t, std::make_integer_sequence<int, kNumCfg - 7>{}); }

}  // namespace nsk
