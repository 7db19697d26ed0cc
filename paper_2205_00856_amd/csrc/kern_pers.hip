// Persistent whole-system kernels (k_system) of uneven batches, for the tile configurations
// they are built for.
#include "kern_table.hpp"
#include "nshaped_kernels.hpp"

namespace nsk {
namespace {
template <int M, int W>
void reg_one(Tables& t) {
  constexpr int I = cfg_index<M, W>();
  static_assert(I >= 0, "a configuration of the row-tile table");
  t.pers[I][nsd::SRC_EXPL] = (const void*)&nsd::k_system<M, W, nsd::SRC_EXPL>;
  t.pers[I][nsd::SRC_EXPL_CT] = (const void*)&nsd::k_system<M, W, nsd::SRC_EXPL_CT>;
  t.pers[I][nsd::SRC_CN] = (const void*)&nsd::k_system<M, W, nsd::SRC_CN>;
}
}  // namespace

void reg_pers(Tables& t) {
  reg_one<4, 2>(t);
  reg_one<4, 4>(t);
  reg_one<4, 8>(t);
  reg_one<8, 2>(t);
  reg_one<8, 4>(t);
}

}  // namespace nsk
