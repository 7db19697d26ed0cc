// Row-tile kernels (k_tile) of the solve of explicit a, b, c, d arrays: every tile configuration,
// and the chunked first-level partitions of 8192 and 16384 rows (k_tile_chunk).
#include "kern_table.hpp"
#include "nshaped_kernels.hpp"

namespace nsk {
namespace {
template <int I>
void reg_one(Tables& t) {
  constexpr int M = kCfgs[I].M, W = kCfgs[I].W;
  constexpr int S = nsd::SRC_EXPL;
  t.tile[I][S][nsd::PH_SINGLE] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_SINGLE>;
  t.tile[I][S][nsd::PH_REDUCE] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_REDUCE>;
  t.tile[I][S][nsd::PH_SUBST] = (const void*)&nsd::k_tile<M, W, S, nsd::PH_SUBST>;
}
template <int... I>
void reg_range(Tables& t, std::integer_sequence<int, I...>) {
  (reg_one<I + 0>(t), ...);
}
}  // namespace

void reg_tile_expl(Tables& t) {
  reg_range(t, std::make_integer_sequence<int, kNumCfg - 0>{});
  t.chunk[0][0] = (const void*)&nsd::k_tile_chunk<2, nsd::PH_REDUCE>;
  t.chunk[0][1] = (const void*)&nsd::k_tile_chunk<2, nsd::PH_SUBST>;
  t.chunk[1][0] = (const void*)&nsd::k_tile_chunk<4, nsd::PH_REDUCE>;
  t.chunk[1][1] = (const void*)&nsd::k_tile_chunk<4, nsd::PH_SUBST>;
}

}  // namespace nsk
