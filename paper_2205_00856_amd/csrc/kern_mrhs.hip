// Row-tile kernels of one matrix with several right-hand sides (k_tile_mrhs, explicit a, b, c
// shared by the batch): the configurations the plans of such batches use.
#include "kern_table.hpp"
#include "nshaped_kernels.hpp"

namespace nsk {
namespace {
template <int M, int W>
void reg_one(Tables& t) {
  constexpr int I = cfg_index<M, W>();
  static_assert(I >= 0, "a configuration of the row-tile table");
  t.mrhs[I][nsd::PH_SINGLE] = (const void*)&nsd::k_tile_mrhs<M, W, nsd::PH_SINGLE>;
  t.mrhs[I][nsd::PH_REDUCE] = (const void*)&nsd::k_tile_mrhs<M, W, nsd::PH_REDUCE>;
  t.mrhs[I][nsd::PH_SUBST] = (const void*)&nsd::k_tile_mrhs<M, W, nsd::PH_SUBST>;
}
}  // namespace

void reg_mrhs(Tables& t) {
  reg_one<2, 1>(t);
  reg_one<2, 2>(t);
  reg_one<2, 4>(t);
  reg_one<4, 1>(t);
  reg_one<4, 2>(t);
  reg_one<4, 4>(t);
  reg_one<4, 8>(t);
  reg_one<8, 4>(t);
}

}  // namespace nsk
