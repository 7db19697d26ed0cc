// Resident propagation kernels (k_resident): every step of a Crank-Nicolson propagation of one
// system in one launch, for the tile configurations of kResCfgs, with real potentials and with
// an absorbing part.
#include "kern_table.hpp"
#include "nshaped_kernels.hpp"

namespace nsk {
namespace {
template <int I>
void reg_one(Tables& t) {
  constexpr int M = kResCfgs[I].M, W = kResCfgs[I].W;
  t.res[I][0] = (const void*)&nsd::k_resident<M, W, nsd::SRC_CN>;
  t.res[I][1] = (const void*)&nsd::k_resident<M, W, nsd::SRC_CNW>;
}
template <int... I>
void reg_range(Tables& t, std::integer_sequence<int, I...>) {
  (reg_one<I>(t), ...);
}
}  // namespace

void reg_resident(Tables& t) { reg_range(t, std::make_integer_sequence<int, kNumResCfg>{}); }

}  // namespace nsk
