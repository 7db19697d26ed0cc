// Column kernels (k_cols) of interleaved batches: every column configuration and source.
#include "kern_table.hpp"
#include "nshaped_kernels.hpp"

namespace nsk {
namespace {
template <int I, int S>
void reg_src(Tables& t) {
  constexpr int M = kColCfgs[I].M, W = kColCfgs[I].W;
  t.cols[I][S][nsd::PH_SINGLE] = (const void*)&nsd::k_cols<M, W, S, nsd::PH_SINGLE>;
  t.cols[I][S][nsd::PH_REDUCE] = (const void*)&nsd::k_cols<M, W, S, nsd::PH_REDUCE>;
  t.cols[I][S][nsd::PH_SUBST] = (const void*)&nsd::k_cols<M, W, S, nsd::PH_SUBST>;
}
template <int I>
void reg_one(Tables& t) {
  reg_src<I, nsd::SRC_EXPL>(t);
  reg_src<I, nsd::SRC_EXPL_CT>(t);
  reg_src<I, nsd::SRC_CN>(t);
}
template <int... I>
void reg_range(Tables& t, std::integer_sequence<int, I...>) {
  (reg_one<I>(t), ...);
}
}  // namespace

void reg_cols(Tables& t) {
  reg_range(t, std::make_integer_sequence<int, kNumColCfg>{});
  // the partial waves' field coupling: the default column tile (64 rows, 16 per lane)
  reg_src<col_cfg_index<16, 4>(), nsd::SRC_LCOUP>(t);
}

}  // namespace nsk
