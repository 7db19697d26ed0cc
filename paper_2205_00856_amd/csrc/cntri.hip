// Host runtime and C ABI of the N-shaped partition Crank-Nicolson solver (gfx950).
// The ABI is declared and documented in include/cntri.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cntri.h"
#include "kern_table.hpp"
#include "nshaped_kernels.hpp"

using nsd::cd;
using nsd::KArgs;

// The kernel entry addresses, filled once (on first use) by the kern_*.hip units.
nsk::Tables& nsk::tables() {
  static Tables t = [] {
    Tables x{};
    reg_tile_expl(x);
    reg_tile_ct(x);
    reg_tile_cn_lo(x);
    reg_tile_cn_hi(x);
    reg_tile_cnw(x);
    reg_tile_slots(x);
    reg_cols(x);
    reg_pers(x);
    reg_mrhs(x);
    reg_aux(x);
    reg_resident(x);
    return x;
  }();
  return t;
}

namespace {

// ----------------------------------------------------------------------- kernel table
using nsk::Cfg;
using nsk::kCfgs;
using nsk::kColCfgs;
using nsk::kNumCfg;
using nsk::kNumColCfg;

const void* const (&g_kern)[kNumCfg][nsk::kNumSrc][nsk::kNumPh] = nsk::tables().tile;
const void* const (&g_pers)[kNumCfg][nsk::kNumSrc] = nsk::tables().pers;
const void* const (&g_cols)[kNumColCfg][nsk::kNumSrc][3] = nsk::tables().cols;
const void* aux_fn(int k) { return nsk::tables().aux[k]; }
const void* const (&g_mrhs)[kNumCfg][3] = nsk::tables().mrhs;

int col_cfg(int64_t T, int M) {
  for (int i = 0; i < kNumColCfg; ++i)
    if ((int64_t)kColCfgs[i].M * kColCfgs[i].W == T && (M == 0 || kColCfgs[i].M == M)) return i;
  return -1;
}

// CN_LOG=1: every new plan is described on stderr when it is built
bool log_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_LOG");
    return e && e[0] == '1';
  }();
  return on;
}

// column kernels for interleaved batches (CN_COLS=0 turns them off)
bool cols_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_COLS");
    return !(e && e[0] == '0');
  }();
  return on;
}

int find_cfg(int64_t T, int M) {
  for (int i = 0; i < kNumCfg; ++i)
    if (kCfgs[i].T() == T && kCfgs[i].M == M) return i;
  return -1;
}

constexpr int64_t kSingleMax = 4096;  // largest tile that solves a whole system in one pass

// First-level partitions of the explicit solve beyond one workgroup's tile: chunks of 4096 rows
// (k_tile_chunk), 2 for 8192 rows and 4 for 16384; 0 for other sizes.
int chunks_of(int64_t partition) {
  return partition == 8192 ? 2 : partition == 16384 ? 4 : 0;
}

// persistent launch for uneven batches (CN_PERSIST=0 turns it off)
bool persist_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_PERSIST");
    return !(e && e[0] == '0');
  }();
  return on;
}

// reverse mode with the segment recompute overlapped on a second stream (CN_BWD_OVERLAP=0
// turns it off)
bool bwd_overlap_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_BWD_OVERLAP");
    return !(e && e[0] == '0');
  }();
  return on;
}

// second passes take their tiles in reverse order (CN_REV=0 turns it off) when the level holds
// at least 2^21 rows; smaller levels stay in the XCDs' L2 between the passes anyway
bool rev_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_REV");
    return !(e && e[0] == '0');
  }();
  return on;
}
int rev_for(int64_t rows) { return (rev_enabled() && rows >= ((int64_t)1 << 21)) ? 1 : 0; }

// one matrix with several right-hand sides through k_tile_mrhs, the matrix loaded once per tile
// (CN_MRHS=0 turns it off: every right-hand side then has workgroups of its own)
bool mrhs_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_MRHS");
    return !(e && e[0] == '0');
  }();
  return on;
}

// Right-hand sides per workgroup of a k_tile_mrhs launch over K tiles of a batch: as many as
// keep at least 1024 workgroups (four per CU) in the launch.
int64_t mrhs_per_wg(int64_t K, int64_t batch) {
  const int64_t groups = std::min<int64_t>(batch, std::max<int64_t>(1, (1024 + K - 1) / K));
  return (batch + groups - 1) / groups;
}

// XCD-contiguous order of whole-system workgroups (CN_XCD_REMAP=0 turns it off)
bool xcd_remap_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_XCD_REMAP");
    return !(e && e[0] == '0');
  }();
  return on;
}

// Workgroup configuration for a system that fits one tile: the smallest tile that holds it.
int single_cfg(int64_t n) {
  if (n <= 128) return find_cfg(128, 2);
  if (n <= 256) return find_cfg(256, 4);
  if (n <= 512) return find_cfg(512, 4);
  if (n <= 1024) return find_cfg(1024, 4);
  if (n <= 2048) return find_cfg(2048, 8);
  return find_cfg(4096, 8);
}

// ------------------------------------------------------------------------------- plans
enum class Src { EXPL = nsd::SRC_EXPL, CT = nsd::SRC_EXPL_CT, CN = nsd::SRC_CN, CNW = nsd::SRC_CNW };

// steps with an absorbing potential take the fused kernels (CN_ABSORB_FUSED=0 turns them off;
// the steps then run materialised)
bool absorb_fused_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_ABSORB_FUSED");
    return !(e && e[0] == '0');
  }();
  return on;
}

struct Launch {
  const void* fn;
  dim3 grid;
  int threads;
  KArgs a;
  int level;  // 1 = the caller's system
  int src, ph, cfg;
  // table offsets (bytes into plan tables) or -1
  int64_t t_offs = -1, t_tbase = -1, t_wgs = -1, t_wgt = -1, t_queue = -1;
  // workspace offsets (bytes) or -1
  int64_t o_sU = -1, o_sD = -1, o_oU = -1, o_oD = -1, o_x = -1, o_psi_if = -1, o_hout = -1,
          o_hin = -1;
  int64_t o_hout2 = -1;  // second edge-row array of a Crank-Nicolson first pass (PH_FUSE chains)
};

struct Plan {
  std::vector<Launch> L;
  size_t ws_bytes = 0;
  void* tables = nullptr;
  size_t tables_bytes = 0;
  std::string desc;
  int64_t span = 0;  // element extent of the caller's arrays
  int64_t rows = 0;  // total rows
  int64_t o_aux = -1;   // workspace for an extra state vector (adjoint step)
  int64_t o_part = -1;  // workspace for per-block partial sums
  int64_t nparts = 0;
  int64_t ntiles1 = 0;  // level-1 tiles of a uniform CN plan (partial sums of the adjoint)
  std::vector<char> host_tab;  // no-allocation plans: the tables, copied into scratch per call
  ~Plan() {
    if (tables) (void)hipFree(tables);
  }
};

struct Knobs {
  int64_t partition = 0;
  int rpt = 0;
  int shared = 0;  // level-1 systems share system 0's coefficients
  int levels = 0;  // > 0: serial RS stage on the reduced systems left after this many levels
};

struct Builder {
  std::vector<char> tab;
  size_t ws = 0;
  std::string desc;
  int64_t add_tab(const void* p, size_t bytes) {
    size_t off = (tab.size() + 255) & ~size_t(255);
    tab.resize(off + bytes);
    if (bytes) memcpy(tab.data() + off, p, bytes);
    return (int64_t)off;
  }
  int64_t add_ws(size_t bytes) {
    size_t off = (ws + 255) & ~size_t(255);
    ws = off + std::max<size_t>(bytes, 16);
    return (int64_t)off;
  }
};

int num_cus() {
  static int cus = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return v > 0 ? v : 256;
  }();
  return cus;
}

struct BatchDesc {
  bool uneven = false;
  int64_t n = 0, batch = 0, es = 1, bs = 1;
  std::vector<int64_t> offs;
};

int multi_cfg(int64_t n, int64_t batch, const Knobs& k, int level, int src) {
  if (level == 1 && k.partition > 0) {
    int M = k.rpt > 0 ? k.rpt : (k.partition >= 512 ? 8 : 4);
    int ci = find_cfg(k.partition, M);
    if (ci < 0) ci = find_cfg(k.partition, 4);
    if (ci < 0) ci = find_cfg(k.partition, 8);
    if (ci < 0) ci = find_cfg(k.partition, 2);
    if (ci < 0) ci = find_cfg(k.partition, 1);
    return ci;
  }
  // Crank-Nicolson lines with enough rows for 512 tiles of 2048: 8 rows per lane, whose
  // substitution runs along the RD rows (measured 10% faster per step at 2^20 and 2^24 rows;
  // with an absorbing potential 20% faster at 2^24 than 1024-row tiles of 4 rows per lane)
  if (level == 1 && nsd::cn_src(src) && k.rpt == 0 && batch * ((n + 2047) / 2048) >= 512)
    return find_cfg(2048, 8);
  // enough tiles to fill the chip (>= 4 workgroups per CU when the system allows it)
  const int64_t target = 1024;
  int64_t T = 1024;
  while (T > 256 && batch * ((n + T - 1) / T) < target) T /= 2;
  int M = (level == 1 && k.rpt > 0) ? k.rpt : 4;
  int ci = find_cfg(T, M);
  if (ci < 0) ci = find_cfg(T, 4);
  return ci;
}

void add_launch(std::vector<Launch>& L, int ci, int src, int ph, dim3 grid, int level,
                const KArgs& a) {
  Launch l;
  l.fn = g_kern[ci][src][ph];
  l.grid = grid;
  l.threads = 64 * kCfgs[ci].W;
  l.a = a;
  l.level = level;
  l.src = src;
  l.ph = ph;
  l.cfg = ci;
  L.push_back(l);
}

std::string cfg_str(int ci) {
  char s[64];
  snprintf(s, sizeof(s), "T=%lld(M=%d,W=%d)", (long long)kCfgs[ci].T(), kCfgs[ci].M, kCfgs[ci].W);
  return s;
}

// The RS stage of Table 1 on the reduced systems of a level, serially (Thomas's elimination, one
// thread per system): the top of a plan whose nesting depth the caller fixed (cn_layout.levels).
// bd: the reduced systems (uneven: offsets over the slot rows); x goes to workspace offset o_x.
void plan_serial_rs(Builder& B, std::vector<Launch>& L, const BatchDesc& bd, int level,
                    int64_t o_sU, int64_t o_sD, int64_t o_x) {
  const int64_t rows = bd.offs[bd.batch];
  Launch l;
  l.fn = aux_fn(nsk::AUX_RS_SERIAL);
  l.grid = dim3((unsigned)((bd.batch + 63) / 64));
  l.threads = 64;
  l.a = KArgs{};
  l.a.vscale = 1.0;
  l.a.batch = bd.batch;
  l.level = level;
  l.src = nsd::SRC_SLOTS;
  l.ph = nsd::PH_SINGLE;
  l.cfg = -1;
  l.t_offs = B.add_tab(bd.offs.data(), (bd.batch + 1) * sizeof(int64_t));
  l.o_sU = o_sU;
  l.o_sD = o_sD;
  l.o_x = o_x;
  l.o_oU = B.add_ws(rows * sizeof(cd));  // eliminated super-diagonal c' per row
  l.o_oD = B.add_ws(rows * sizeof(cd));  // eliminated right-hand side d' per row
  L.push_back(l);
  char line[128];
  snprintf(line, sizeof(line), "L%d serial RS systems=%lld rows=%lld; ", level,
           (long long)bd.batch, (long long)rows);
  B.desc += line;
}

void plan_level(Builder& B, std::vector<Launch>& L, const BatchDesc& bd, int src, int level,
                int64_t o_sU, int64_t o_sD, int64_t o_x, const Knobs& kn);

// The reduced systems of a uniform batch split into K tiles per system: batch systems of K
// rows each, their slots at system * K + tile.  As a uniform batch (element stride 1, batch
// stride K) the level's launches find a system's slots from its index, with no table lookup;
// the serial RS stage of a fixed nesting depth takes them as an uneven batch of equal lengths.
void plan_reduced_uniform(Builder& B, std::vector<Launch>& L, int64_t batch, int64_t K, int level,
                          int64_t oU, int64_t oD, int64_t oP, const Knobs& kn) {
  BatchDesc ib;
  if (kn.levels > 0 && level >= kn.levels) {
    ib.uneven = true;
    ib.batch = batch;
    ib.offs.resize(batch + 1);
    for (int64_t s = 0; s <= batch; ++s) ib.offs[s] = s * K;
    plan_serial_rs(B, L, ib, level + 1, oU, oD, oP);
    return;
  }
  ib.uneven = false;
  ib.n = K;
  ib.batch = batch;
  ib.es = 1;
  ib.bs = K;
  plan_level(B, L, ib, nsd::SRC_SLOTS, level + 1, oU, oD, oP, kn);
}

// Appends the launches that solve one level; x goes to the caller (level 1) or to workspace
// offset o_x.  At level >= 2 the source is the slot arrays at (o_sU, o_sD).
void plan_level(Builder& B, std::vector<Launch>& L, const BatchDesc& bd, int src, int level,
                int64_t o_sU, int64_t o_sD, int64_t o_x, const Knobs& kn) {
  KArgs base{};
  base.vscale = 1.0;
  base.cshared = (level == 1) ? kn.shared : 0;
  auto set_common = [&](Launch& l) {
    l.o_sU = o_sU;
    l.o_sD = o_sD;
    l.o_x = o_x;
  };
  char line[256];
  if (!bd.uneven) {
    const int64_t n = bd.n, batch = bd.batch;
    if (bd.bs == 1 && batch >= 64 && bd.es >= batch && src != nsd::SRC_SLOTS &&
        src != nsd::SRC_CNW && cols_enabled() && !kn.shared) {
      int cc = -1;
      if (level == 1 && kn.partition > 0) cc = col_cfg(kn.partition, kn.rpt);
      if (cc < 0) cc = col_cfg(64, 16);
      const int64_t T = (int64_t)kColCfgs[cc].M * kColCfgs[cc].W;
      const int64_t K = (n + T - 1) / T, G = K * batch;
      const unsigned gy = (unsigned)((batch + 63) / 64);
      KArgs a = base;
      a.n = n;
      a.ntiles = K;
      a.es = bd.es;
      a.bs = bd.bs;
      a.batch = batch;
      a.nitems = (int)std::min<int64_t>(G, INT32_MAX);
      auto add_col = [&](int ph) {
        Launch l;
        l.fn = g_cols[cc][src][ph];
        l.grid = dim3((unsigned)(K * gy));
        l.threads = 64 * kColCfgs[cc].W;
        l.a = a;
              l.level = level;
        l.src = src;
        l.ph = ph;
        l.cfg = -1;
        L.push_back(l);
        set_common(L.back());
      };
      char cs[96];
      snprintf(cs, sizeof(cs), "T=%lld(M=%d,W=%d)", (long long)T, kColCfgs[cc].M, kColCfgs[cc].W);
      if (K == 1) {
        add_col(nsd::PH_SINGLE);
        snprintf(line, sizeof(line), "L%d columns single %s n=%lld batch=%lld; ", level, cs,
                 (long long)n, (long long)batch);
        B.desc += line;
        return;
      }
      const int64_t oU = B.add_ws(3 * G * sizeof(cd)), oD = B.add_ws(3 * G * sizeof(cd));
      const int64_t oP = B.add_ws(G * sizeof(cd));
      const int64_t oH = nsd::halo_src(src) ? B.add_ws(2 * G * sizeof(cd)) : -1;
      snprintf(line, sizeof(line), "L%d columns multi %s n=%lld batch=%lld tiles=%lld; ", level, cs,
               (long long)n, (long long)batch, (long long)K);
      B.desc += line;
      add_col(nsd::PH_REDUCE);
      L.back().o_oU = oU;
      L.back().o_oD = oD;
      L.back().o_hout = oH;
      plan_reduced_uniform(B, L, batch, K, level, oU, oD, oP, kn);
      add_col(nsd::PH_SUBST);
      L.back().a.rev = rev_for(n * batch);
      L.back().o_psi_if = oP;
      L.back().o_hin = oH;
      return;
    }
    int ci_single = -1;
    if (level == 1 && kn.partition > 0) {
      if (n <= kn.partition) ci_single = multi_cfg(n, batch, kn, level, src);
    } else if (n <= kSingleMax && (batch >= 64 || n <= 1024 || level > 1)) {
      ci_single = single_cfg(n);
      // reduced systems of up to 64 joints: one row per lane, no idle lanes (the ADI y-sweep's
      // 4096 systems of 64 joints: 0.5 % of the step faster than 2 rows on half the lanes)
      if (src == nsd::SRC_SLOTS && n <= 64) ci_single = find_cfg(64, 1);
    }
    // one matrix, several right-hand sides: k_tile_mrhs launches (grid y = groups of nrhs)
    auto mrhs_of = [&](int ci) {
      return (level == 1 && kn.shared && src == nsd::SRC_EXPL && batch >= 2 && mrhs_enabled() &&
              g_mrhs[ci][nsd::PH_SINGLE] && g_mrhs[ci][nsd::PH_REDUCE] && g_mrhs[ci][nsd::PH_SUBST]);
    };
    if (ci_single >= 0) {
      const int ci = ci_single;
      KArgs a = base;
      a.n = n;
      a.ntiles = 1;
      a.es = bd.es;
      a.bs = bd.bs;
      a.xcd_remap = xcd_remap_enabled() ? 1 : 0;
      if (mrhs_of(ci)) {
        a.xcd_remap = 0;
        a.batch = batch;
        a.nrhs = (int)mrhs_per_wg(1, batch);
        const int64_t groups = (batch + a.nrhs - 1) / a.nrhs;
        add_launch(L, ci, src, nsd::PH_SINGLE, dim3(1, (unsigned)groups), level, a);
        L.back().fn = g_mrhs[ci][nsd::PH_SINGLE];
        set_common(L.back());
        snprintf(line, sizeof(line), "L%d single %s n=%lld batch=%lld rhs/wg=%d; ", level,
                 cfg_str(ci).c_str(), (long long)n, (long long)batch, a.nrhs);
        B.desc += line;
        return;
      }
      add_launch(L, ci, src, nsd::PH_SINGLE, dim3(1, (unsigned)batch), level, a);
      set_common(L.back());
      snprintf(line, sizeof(line), "L%d single %s n=%lld batch=%lld; ", level, cfg_str(ci).c_str(),
               (long long)n, (long long)batch);
      B.desc += line;
      return;
    }
    // an explicit partition of 8192 or 16384 rows: chunked partitions (two-pass, the second
    // pass reading each chunk twice)
    if (level == 1 && src == nsd::SRC_EXPL && chunks_of(kn.partition) > 0 && !kn.shared) {
      const int C = chunks_of(kn.partition);
      const int ci = find_cfg(4096, 8);
      const int64_t T = kn.partition;
      const int64_t K = (n + T - 1) / T, G = K * batch;
      const int64_t oU = B.add_ws(3 * G * sizeof(cd)), oD = B.add_ws(3 * G * sizeof(cd));
      const int64_t oP = B.add_ws(G * sizeof(cd));
      KArgs a = base;
      a.n = n;
      a.ntiles = K;
      a.es = bd.es;
      a.bs = bd.bs;
      snprintf(line, sizeof(line), "L%d multi T=%lld(%d chunks of T=4096(M=8,W=8)) n=%lld "
               "batch=%lld tiles=%lld; ", level, (long long)T, C, (long long)n,
               (long long)batch, (long long)K);
      B.desc += line;
      add_launch(L, ci, src, nsd::PH_REDUCE, dim3((unsigned)K, (unsigned)batch), level, a);
      L.back().fn = nsk::tables().chunk[C == 4][0];
      set_common(L.back());
      L.back().o_oU = oU;
      L.back().o_oD = oD;
      plan_reduced_uniform(B, L, batch, K, level, oU, oD, oP, kn);
      add_launch(L, ci, src, nsd::PH_SUBST, dim3((unsigned)K, (unsigned)batch), level, a);
      L.back().fn = nsk::tables().chunk[C == 4][1];
      set_common(L.back());
      L.back().o_psi_if = oP;
      return;
    }
    int ci = multi_cfg(n, batch, kn, level, src);
    const int64_t T = kCfgs[ci].T();
    const int64_t K = (n + T - 1) / T, G = K * batch;
    const int64_t oU = B.add_ws(3 * G * sizeof(cd)), oD = B.add_ws(3 * G * sizeof(cd));
    const int64_t oP = B.add_ws(G * sizeof(cd));
    const int64_t oH = nsd::cn_src(src) ? B.add_ws(2 * G * sizeof(cd)) : -1;
    const int64_t oH2 = nsd::cn_src(src) ? B.add_ws(2 * G * sizeof(cd)) : -1;
    KArgs a = base;
    a.n = n;
    a.ntiles = K;
    a.es = bd.es;
    a.bs = bd.bs;
    const bool mr = mrhs_of(ci);
    unsigned gy = (unsigned)batch;
    if (mr) {
      a.batch = batch;
      a.nrhs = (int)mrhs_per_wg(K, batch);
      gy = (unsigned)((batch + a.nrhs - 1) / a.nrhs);
      snprintf(line, sizeof(line), "L%d multi %s n=%lld batch=%lld tiles=%lld rhs/wg=%d; ",
               level, cfg_str(ci).c_str(), (long long)n, (long long)batch, (long long)K, a.nrhs);
    } else {
      snprintf(line, sizeof(line), "L%d multi %s n=%lld batch=%lld tiles=%lld; ", level,
               cfg_str(ci).c_str(), (long long)n, (long long)batch, (long long)K);
    }
    B.desc += line;
    add_launch(L, ci, src, nsd::PH_REDUCE, dim3((unsigned)K, gy), level, a);
    if (mr) L.back().fn = g_mrhs[ci][nsd::PH_REDUCE];
    set_common(L.back());
    L.back().o_oU = oU;
    L.back().o_oD = oD;
    L.back().o_hout = oH;
    L.back().o_hout2 = oH2;
    plan_reduced_uniform(B, L, batch, K, level, oU, oD, oP, kn);
    add_launch(L, ci, src, nsd::PH_SUBST, dim3((unsigned)K, gy), level, a);
    if (mr) L.back().fn = g_mrhs[ci][nsd::PH_SUBST];
    L.back().a.rev = batch == 1 ? rev_for(n) : 0;  // one-dimensional grids only
    set_common(L.back());
    L.back().o_psi_if = oP;
    L.back().o_hin = oH;
    return;
  }
  // uneven batch
  const int64_t batch = bd.batch;
  const int64_t t_offs = B.add_tab(bd.offs.data(), (batch + 1) * sizeof(int64_t));
  int64_t handled = 0;  // systems up to this length went to the persistent launch
  // with an explicit partition: one persistent launch, whole systems from a device queue,
  // longest first (configurations without a persistent kernel use T = 1024, M = 4; a source
  // without persistent kernels, such as the column-only field coupling, takes the other path)
  int pci = -1;
  if (level == 1 && src != nsd::SRC_SLOTS && src != nsd::SRC_CNW && kn.partition > 0 &&
      persist_enabled()) {
    pci = find_cfg(kn.partition, kn.rpt > 0 ? kn.rpt : 4);
    if (pci >= 0 && !g_pers[pci][src]) pci = -1;
    if (pci < 0) pci = find_cfg(1024, 4);
    if (!g_pers[pci][src]) pci = -1;
  }
  if (pci >= 0) {
    const int ci = pci;
    const int64_t T = kCfgs[ci].T();
    handled = nsd::kMaxSysTiles * T;
    std::vector<int> sys;
    BatchDesc rest;
    rest.uneven = true;
    rest.batch = batch;
    rest.offs.assign(batch + 1, 0);
    int64_t rest_rows = 0;
    for (int64_t s = 0; s < batch; ++s) {
      const int64_t len = bd.offs[s + 1] - bd.offs[s];
      if (len > 0 && len <= nsd::kMaxSysTiles * T) sys.push_back((int)s);
    }
    std::stable_sort(sys.begin(), sys.end(), [&](int p, int q) {
      return bd.offs[p + 1] - bd.offs[p] > bd.offs[q + 1] - bd.offs[q];
    });
    if (!sys.empty()) {
      int per_cu = 1;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, g_pers[ci][src], 64 * kCfgs[ci].W,
                                                       0) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();  // the query's failure is handled here: leave no error behind
        per_cu = 1;
      }
      const int64_t grid = std::min<int64_t>((int64_t)per_cu * num_cus(), (int64_t)sys.size());
      Launch l;
      l.fn = g_pers[ci][src];
      l.grid = dim3((unsigned)grid);
      l.threads = 64 * kCfgs[ci].W;
      l.a = base;
      l.a.nitems = (int)sys.size();
      l.level = level;
      l.src = src;
      l.ph = -1;
      l.cfg = ci;
      l.t_offs = t_offs;
      l.t_wgs = B.add_tab(sys.data(), sys.size() * sizeof(int));
      const int zero2[2] = {0, 0};
      l.t_queue = B.add_tab(zero2, sizeof(zero2));
      L.push_back(l);
      set_common(L.back());
      snprintf(line, sizeof(line), "L%d persistent %s systems=%zu grid=%lld; ", level,
               cfg_str(ci).c_str(), sys.size(), (long long)grid);
      B.desc += line;
    }
    // systems longer than the in-workgroup limit go through the multi-workgroup path
    bool any_long = false;
    for (int64_t s = 0; s < batch; ++s) {
      const int64_t len = bd.offs[s + 1] - bd.offs[s];
      rest.offs[s + 1] = rest.offs[s];
      if (len > nsd::kMaxSysTiles * T) any_long = true;
    }
    if (!any_long) return;
    (void)rest_rows;
  }
  std::map<int, std::vector<int>> buckets;
  std::vector<int> large;
  for (int64_t s = 0; s < batch; ++s) {
    const int64_t len = bd.offs[s + 1] - bd.offs[s];
    if (len <= 0 || len <= handled) continue;
    if (len <= kSingleMax) {
      buckets[single_cfg(len)].push_back((int)s);
    } else {
      large.push_back((int)s);
    }
  }
  for (auto& kv : buckets) {
    std::vector<int>& sys = kv.second;
    // longest first inside the bucket
    std::stable_sort(sys.begin(), sys.end(), [&](int p, int q) {
      return bd.offs[p + 1] - bd.offs[p] > bd.offs[q + 1] - bd.offs[q];
    });
    std::vector<int> tiles(sys.size(), 0);
    KArgs a = base;
    add_launch(L, kv.first, src, nsd::PH_SINGLE, dim3((unsigned)sys.size()), level, a);
    set_common(L.back());
    L.back().t_offs = t_offs;
    L.back().t_wgs = B.add_tab(sys.data(), sys.size() * sizeof(int));
    L.back().t_wgt = B.add_tab(tiles.data(), tiles.size() * sizeof(int));
    snprintf(line, sizeof(line), "L%d single %s systems=%zu; ", level, cfg_str(kv.first).c_str(),
             sys.size());
    B.desc += line;
  }
  if (large.empty()) return;
  int64_t maxlen = 0, nl = 0;
  for (int s : large) {
    maxlen = std::max(maxlen, bd.offs[s + 1] - bd.offs[s]);
    nl += bd.offs[s + 1] - bd.offs[s];
  }
  // automatic plan of a caller's uneven batch: the long systems are solved two-pass over
  // 2048-row tiles of 8 rows per lane (measured best for lengths up to 65536)
  int ci = (level == 1 && kn.partition == 0 && src != nsd::SRC_SLOTS)
               ? find_cfg(2048, 8)
               : multi_cfg(nl / (int64_t)large.size(), (int64_t)large.size(), kn, level, src);
  const int64_t T = kCfgs[ci].T();
  std::vector<int64_t> tbase(batch + 1, 0);
  std::vector<int> wgs, wgt;
  for (int64_t s = 0; s < batch; ++s) {
    // tiles only for the systems of this launch: longer than one tile and not taken by the
    // persistent launch (an uncounted system's reduced system would be left unwritten)
    const int64_t len = bd.offs[s + 1] - bd.offs[s];
    const int64_t K = (len > kSingleMax && len > handled) ? (len + T - 1) / T : 0;
    tbase[s + 1] = tbase[s] + K;
  }
  // workgroups of the longest systems first
  std::vector<int> order(large);
  std::stable_sort(order.begin(), order.end(), [&](int p, int q) {
    return bd.offs[p + 1] - bd.offs[p] > bd.offs[q + 1] - bd.offs[q];
  });
  for (int s : order)
    for (int64_t t = 0; t < tbase[s + 1] - tbase[s]; ++t) {
      wgs.push_back(s);
      wgt.push_back((int)t);
    }
  const int64_t G = tbase[batch];
  const int64_t oU = B.add_ws(3 * G * sizeof(cd)), oD = B.add_ws(3 * G * sizeof(cd));
  const int64_t oP = B.add_ws(G * sizeof(cd));
  const int64_t oH = nsd::cn_src(src) ? B.add_ws(2 * G * sizeof(cd)) : -1;
  const int64_t oH2 = nsd::cn_src(src) ? B.add_ws(2 * G * sizeof(cd)) : -1;
  const int64_t t_tb = B.add_tab(tbase.data(), (batch + 1) * sizeof(int64_t));
  const int64_t t_s = B.add_tab(wgs.data(), wgs.size() * sizeof(int));
  const int64_t t_t = B.add_tab(wgt.data(), wgt.size() * sizeof(int));
  snprintf(line, sizeof(line), "L%d multi %s systems=%zu tiles=%lld; ", level, cfg_str(ci).c_str(),
           large.size(), (long long)G);
  B.desc += line;
  KArgs a = base;
  add_launch(L, ci, src, nsd::PH_REDUCE, dim3((unsigned)wgs.size()), level, a);
  set_common(L.back());
  L.back().t_offs = t_offs;
  L.back().t_tbase = t_tb;
  L.back().t_wgs = t_s;
  L.back().t_wgt = t_t;
  L.back().o_oU = oU;
  L.back().o_oD = oD;
  L.back().o_hout = oH;
  L.back().o_hout2 = oH2;
  BatchDesc ib;
  ib.uneven = true;
  ib.batch = batch;
  ib.offs = tbase;
  if (kn.levels > 0 && level >= kn.levels)
    plan_serial_rs(B, L, ib, level + 1, oU, oD, oP);
  else
    plan_level(B, L, ib, nsd::SRC_SLOTS, level + 1, oU, oD, oP, kn);
  add_launch(L, ci, src, nsd::PH_SUBST, dim3((unsigned)wgs.size()), level, a);
  set_common(L.back());
  L.back().a.rev = rev_for(nl);
  L.back().t_offs = t_offs;
  L.back().t_tbase = t_tb;
  L.back().t_wgs = t_s;
  L.back().t_wgt = t_t;
  L.back().o_psi_if = oP;
  L.back().o_hin = oH;
}

}  // namespace

// ------------------------------------------------------------------------------- handle
struct cn_handle_s {
  int device = 0;
  void* ws = nullptr;
  size_t ws_size = 0;
  int* status = nullptr;
  // done counts of the fused passes that solve their reduced system themselves, one for chains
  // on ws and one (at +32) for chains on ws2; zero between launches (same allocation as status)
  int* sync = nullptr;
  std::map<std::string, std::unique_ptr<Plan>> plans;
  std::map<std::string, std::string> tuned;  // automatic layout key -> key of the tuned plan
  double* rows_buf = nullptr;  // per-step partial sums of one checkpoint segment
  size_t rows_cap = 0;         // doubles
  // reverse mode: the recompute of the next checkpoint segment runs on a second stream (default
  // priority) with a workspace and a segment buffer of its own
  hipStream_t aux = nullptr;
  hipEvent_t ev[5] = {};
  void* ws2 = nullptr;
  size_t ws2_size = 0;
  void* seg2 = nullptr;
  size_t seg2_bytes = 0;
  // materialised a, b, c, d of steps with an absorbing potential
  void* mat = nullptr;
  size_t mat_size = 0;
  // partial-wave step: centrifugal potentials, then the field part's a, b, c, d
  void* rad = nullptr;
  size_t rad_size = 0;
  // Once a call of this handle has been captured into a HIP graph, the graph holds the device
  // addresses of the handle's buffers: a buffer replaced by a larger one is then kept here
  // until cn_destroy instead of being freed.
  bool captured = false;
  std::vector<void*> retired;
  // cn_tridiag_solve_noalloc: this device's address of the fixed scratch array, and the plans
  // of that entry point (their tables live in host memory and are copied into the array)
  char* scratch = nullptr;
  std::map<std::string, std::unique_ptr<Plan>> static_plans;
  // persistent autotune cache (cn_tune_cache): file path and entries, layout class -> "T,M"
  std::string cache_path;
  std::map<std::string, std::string> cache;
  // resident propagation: slots, edge rows and joint values of its tiles, then the field
  void* res = nullptr;
  size_t res_size = 0;
  // plan log (cn_profile): HIP events around every launch of run_plan, with a label each
  bool profiling = false;
  struct Rec {
    std::string label;
    hipEvent_t e0, e1;
  };
  std::vector<Rec> recs;
};

namespace {

#define HIP_TRY(expr)                        \
  do {                                       \
    if ((expr) != hipSuccess) return CN_ERR_HIP; \
  } while (0)

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st != hipStreamCaptureStatusNone;
}

// ------------------------------------------------------------ fixed scratch (no allocation)
// Device memory of cn_tridiag_solve_noalloc: the plan tables (offsets, launch lists) at the
// start, then the workspace (slots, reduced solutions).  One copy per GPU, held until the
// process ends.  In host code `scratch` is only a host-side stand-in for the symbol: its device
// address on each GPU comes from hipGetSymbolAddress (scratch_setup) and only that address is
// passed to kernels and copies.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[kMaxDevices] = {};

// Resolves this device's address of `scratch` once per device; `device` must be current.
cn_status scratch_setup(int device, char** addr) {
  if (device < 0 || device >= kMaxDevices) return CN_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CN_ERR_HIP;
    g_scratch_addr[device] = (char*)p;
  }
  *addr = g_scratch_addr[device];
  return CN_OK;
}

// Replaces handle buffer *p (size *bytes) by a new allocation of `need` bytes.  The old buffer
// is freed (after the device is idle) unless a graph captured on this handle may still use it;
// then it is retired until cn_destroy.  Never called during capture.
cn_status regrow(cn_handle_t h, void** p, size_t* bytes, size_t need) {
  if (*p) {
    if (h->captured) {
      h->retired.push_back(*p);
    } else {
      if (hipDeviceSynchronize() != hipSuccess) return CN_ERR_HIP;
      (void)hipFree(*p);
    }
  }
  *p = nullptr;
  *bytes = 0;
  if (hipMalloc(p, need) != hipSuccess) {
    *p = nullptr;
    return CN_ERR_NO_MEMORY;
  }
  *bytes = need;
  return CN_OK;
}

cn_status validate(const cn_layout* L, int64_t& rows, int64_t& span) {
  if (!L) return CN_ERR_INVALID_ARG;
  if (L->batch < 1) return CN_ERR_INVALID_ARG;
  if (L->partition != 0) {
    const int64_t p = L->partition;
    if (p < 32 || p > 16384 || (p & (p - 1))) return CN_ERR_INVALID_ARG;
  }
  if (L->rows_per_thread != 0 && L->rows_per_thread != 2 && L->rows_per_thread != 4 &&
      L->rows_per_thread != 8 && L->rows_per_thread != 16)
    return CN_ERR_INVALID_ARG;
  if (L->shared_coefficients != 0 && L->shared_coefficients != 1) return CN_ERR_INVALID_ARG;
  if (L->levels < 0 || L->levels > 8) return CN_ERR_INVALID_ARG;
  if (L->offsets && L->shared_coefficients) return CN_ERR_UNSUPPORTED;
  if (L->offsets) {
    if (L->offsets[0] != 0) return CN_ERR_INVALID_ARG;
    for (int64_t s = 0; s < L->batch; ++s)
      if (L->offsets[s + 1] < L->offsets[s]) return CN_ERR_INVALID_ARG;
    rows = span = L->offsets[L->batch];
    if (rows < 1) return CN_ERR_INVALID_ARG;
    return CN_OK;
  }
  if (L->n < 1 || L->elem_stride < 1 || L->batch_stride < 1) return CN_ERR_INVALID_ARG;
  const int64_t n = L->n, B = L->batch, es = L->elem_stride, bs = L->batch_stride;
  // systems must not share elements: either each system lies inside one batch_stride period,
  // or the systems interleave inside one elem_stride period
  const bool ok = (B == 1) || (bs >= (n - 1) * es + 1) || (es >= (B - 1) * bs + 1);
  if (!ok) return CN_ERR_INVALID_ARG;
  if (n > (int64_t)1 << 40 || B > (int64_t)1 << 31) return CN_ERR_UNSUPPORTED;
  rows = n * B;
  span = (B - 1) * bs + (n - 1) * es + 1;
  return CN_OK;
}

std::string plan_key(const cn_layout* L, int src) {
  std::string k;
  char buf[160];
  snprintf(buf, sizeof(buf), "%d|%lld|%lld|%lld|%lld|%d|%d|%d|%d|", src, (long long)L->n,
           (long long)L->batch, (long long)L->elem_stride, (long long)L->batch_stride,
           L->partition, L->rows_per_thread, L->shared_coefficients, L->levels);
  k = buf;
  if (L->offsets) {
    k += "U";
    k.append(reinterpret_cast<const char*>(L->offsets), (L->batch + 1) * sizeof(int64_t));
  }
  return k;
}

// Builds the launches of a plan for this layout on the host (no device access).  tab receives
// the plan's device tables (offsets, launch lists, queue counters); adjoint_ws adds the
// workspace of cn_step_adjoint (Crank-Nicolson plans).
cn_status build_plan(const cn_layout* L, int src, bool adjoint_ws, Plan& P,
                     std::vector<char>& tab) {
  int64_t rows = 0, span = 0;
  cn_status st = validate(L, rows, span);
  if (st != CN_OK) return st;
  Builder B;
  BatchDesc bd;
  if (L->offsets) {
    bd.uneven = true;
    bd.batch = L->batch;
    bd.offs.assign(L->offsets, L->offsets + L->batch + 1);
  } else {
    bd.n = L->n;
    bd.batch = L->batch;
    bd.es = L->elem_stride;
    bd.bs = L->batch_stride;
  }
  Knobs kn;
  kn.partition = L->partition;
  kn.rpt = L->rows_per_thread;
  kn.shared = L->shared_coefficients;
  kn.levels = L->levels;
  if (kn.partition > 0) {
    const bool columns = !L->offsets && L->batch_stride == 1 && L->batch >= 64 &&
                         L->elem_stride >= L->batch && cols_enabled() &&
                         !L->shared_coefficients;
    const int M = kn.rpt > 0 ? kn.rpt : (kn.partition >= 512 ? 8 : 4);
    const bool rows_ok = find_cfg(kn.partition, M) >= 0 || find_cfg(kn.partition, 4) >= 0 ||
                         find_cfg(kn.partition, 8) >= 0 || find_cfg(kn.partition, 2) >= 0 ||
                         find_cfg(kn.partition, 1) >= 0 ||
                         (chunks_of(kn.partition) > 0 && src == nsd::SRC_EXPL && !L->offsets &&
                          !L->shared_coefficients);
    const bool cols_ok = col_cfg(kn.partition, kn.rpt) >= 0;
    if (columns ? !cols_ok : !rows_ok) return CN_ERR_UNSUPPORTED;
  }
  plan_level(B, P.L, bd, src, 1, -1, -1, -1, kn);
  P.span = span;
  P.rows = rows;
  for (const Launch& l : P.L)
    if (!l.fn) return CN_ERR_UNSUPPORTED;  // a configuration without kernels for this source
  if (nsd::cn_src(src) && adjoint_ws) {
    P.o_aux = B.add_ws(rows * sizeof(cd) + 16);
    P.nparts = (rows + 255) / 256;
    P.o_part = B.add_ws((rows / 64 + 64) * sizeof(double));
    for (const Launch& l : P.L)
      if (l.level == 1 && (l.ph == nsd::PH_SINGLE || l.ph == nsd::PH_SUBST))
        P.ntiles1 = l.a.nitems > 0 ? (int64_t)l.a.nitems : (int64_t)l.grid.x * l.grid.y;
  }
  P.ws_bytes = B.ws;
  P.desc = B.desc;
  tab.swap(B.tab);
  return CN_OK;
}

// Points the launches of a plan at its tables, stored at device address tb.
void bind_tables(Plan& P, char* tb) {
  for (Launch& l : P.L) {
    if (l.t_offs >= 0) l.a.offs = (const int64_t*)(tb + l.t_offs);
    if (l.t_tbase >= 0) l.a.tbase = (const int64_t*)(tb + l.t_tbase);
    if (l.t_wgs >= 0) l.a.wg_sys = (const int*)(tb + l.t_wgs);
    if (l.t_wgt >= 0) l.a.wg_tile = (const int*)(tb + l.t_wgt);
    if (l.t_queue >= 0) l.a.queue = (int*)(tb + l.t_queue);
  }
}

// ------------------------------------------------------------------ autotune cache
// A layout's class for the persistent cache: the device architecture, the source, and the
// layout's shape in power-of-two buckets (rows per system, batch; for uneven batches the total
// rows and the longest system), so that a tuned plan carries over to layouts of the same kind.
std::string arch_name() {
  static const std::string a = [] {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
      return std::string("unknown");
    std::string n = p.gcnArchName;
    const size_t c = n.find(':');
    return c == std::string::npos ? n : n.substr(0, c);
  }();
  return a;
}

int log2_bucket(int64_t v) {
  int b = 0;
  while (((int64_t)1 << (b + 1)) <= v) ++b;
  return b;
}

std::string cache_class(const cn_layout* L, int src) {
  char buf[192];
  if (L->offsets) {
    int64_t maxlen = 0;
    for (int64_t s = 0; s < L->batch; ++s) maxlen = std::max(maxlen, L->offsets[s + 1] - L->offsets[s]);
    snprintf(buf, sizeof(buf), "%s|src%d|uneven|batch2^%d|rows2^%d|max2^%d|levels%d",
             arch_name().c_str(), src, log2_bucket(L->batch), log2_bucket(L->offsets[L->batch]),
             log2_bucket(maxlen), L->levels);
  } else {
    snprintf(buf, sizeof(buf), "%s|src%d|uniform|n2^%d|batch2^%d|es%s|bs%s|shared%d|levels%d",
             arch_name().c_str(), src, log2_bucket(L->n), log2_bucket(L->batch),
             L->elem_stride == 1 ? "1" : "N", L->batch_stride == 1 ? "1" : "N",
             L->shared_coefficients, L->levels);
  }
  return buf;
}

// The cache file is a JSON object of objects (written one entry per line):
//   {"<class>": {"partition": T, "rows_per_thread": M, "ms": t}, ...}
// The reader takes every "<class>": {...} pair whose object holds the two integers.
cn_status cache_load(cn_handle_t h) {
  h->cache.clear();
  FILE* f = fopen(h->cache_path.c_str(), "r");
  if (!f) return CN_OK;  // no file yet
  std::string txt;
  char chunk[4096];
  size_t got;
  while ((got = fread(chunk, 1, sizeof(chunk), f)) > 0) txt.append(chunk, got);
  fclose(f);
  size_t pos = 0;
  for (;;) {
    const size_t q0 = txt.find('"', pos);
    if (q0 == std::string::npos) break;
    const size_t q1 = txt.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    const size_t ob = txt.find_first_not_of(" \t\r\n:", q1 + 1);
    if (ob == std::string::npos || txt[ob] != '{') {  // a key inside an entry: skip it
      pos = q1 + 1;
      continue;
    }
    const size_t cb = txt.find('}', ob);
    if (cb == std::string::npos) break;
    const std::string body = txt.substr(ob, cb - ob);
    int T = 0, M = 0;
    const size_t pp = body.find("\"partition\":"), pm = body.find("\"rows_per_thread\":");
    if (pp != std::string::npos && pm != std::string::npos &&
        sscanf(body.c_str() + pp + 12, "%d", &T) == 1 &&
        sscanf(body.c_str() + pm + 18, "%d", &M) == 1) {
      char v[32];
      snprintf(v, sizeof(v), "%d,%d", T, M);
      h->cache[txt.substr(q0 + 1, q1 - q0 - 1)] = v;
    }
    pos = cb + 1;
  }
  return CN_OK;
}

cn_status cache_store(cn_handle_t h, const std::map<std::string, float>& ms) {
  const std::string tmp = h->cache_path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return CN_ERR_INVALID_ARG;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : h->cache) {
    int T = 0, M = 0;
    sscanf(kv.second.c_str(), "%d,%d", &T, &M);
    auto it = ms.find(kv.first);
    fprintf(f, "  \"%s\": {\"partition\": %d, \"rows_per_thread\": %d, \"ms\": %.6f}%s\n",
            kv.first.c_str(), T, M, it == ms.end() ? -1.0 : (double)it->second,
            ++i < h->cache.size() ? "," : "");
  }
  fprintf(f, "}\n");
  const bool ok = fclose(f) == 0 && rename(tmp.c_str(), h->cache_path.c_str()) == 0;
  return ok ? CN_OK : CN_ERR_INVALID_ARG;
}

cn_status get_plan(cn_handle_t h, const cn_layout* L, int src, hipStream_t s, Plan** out) {
  int64_t rows = 0, span = 0;
  cn_status st = validate(L, rows, span);
  if (st != CN_OK) return st;
  std::string key = plan_key(L, src);
  cn_layout Lc;  // the cached tuned configuration of this layout's class, if any
  {
    auto tk = h->tuned.find(key);
    if (tk != h->tuned.end() && h->plans.count(tk->second)) {
      key = tk->second;
    } else if (!h->cache.empty() && L->partition == 0 && L->rows_per_thread == 0) {
      auto ck = h->cache.find(cache_class(L, src));
      if (ck != h->cache.end()) {
        int T = 0, M = 0;
        if (sscanf(ck->second.c_str(), "%d,%d", &T, &M) == 2 && (T > 0 || M > 0)) {
          Lc = *L;
          Lc.partition = T;
          Lc.rows_per_thread = M;
          int64_t r2 = 0, s2 = 0;
          if (validate(&Lc, r2, s2) == CN_OK) {
            L = &Lc;
            key = plan_key(L, src);
          }
        }
      }
    }
  }
  auto it = h->plans.find(key);
  const bool cap = s != nullptr ? capturing(s) : false;
  if (cap) h->captured = true;
  if (it == h->plans.end()) {
    if (cap) return CN_ERR_NOT_RESERVED;
    std::unique_ptr<Plan> P(new Plan());
    std::vector<char> tab;
    st = build_plan(L, src, true, *P, tab);
    if (st != CN_OK) return st;
    if (!tab.empty()) {
      if (hipMalloc(&P->tables, tab.size()) != hipSuccess) return CN_ERR_NO_MEMORY;
      if (hipMemcpy(P->tables, tab.data(), tab.size(), hipMemcpyHostToDevice) != hipSuccess)
        return CN_ERR_HIP;
      P->tables_bytes = tab.size();
    }
    bind_tables(*P, (char*)P->tables);
    if (log_enabled())
      fprintf(stderr, "cntri: plan for source %d, layout n=%lld batch=%lld%s: %s\n", src,
              (long long)L->n, (long long)L->batch, L->offsets ? " (uneven)" : "",
              P->desc.c_str());
    it = h->plans.emplace(key, std::move(P)).first;
  }
  Plan* P = it->second.get();
  if (P->ws_bytes > h->ws_size) {
    if (cap) return CN_ERR_NOT_RESERVED;
    const cn_status st2 = regrow(h, &h->ws, &h->ws_size, P->ws_bytes);
    if (st2 != CN_OK) return st2;
  }
  *out = P;
  return CN_OK;
}

struct UserArgs {
  const cd *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr;
  const cd* psi = nullptr;
  const cd* rhs = nullptr;
  const double* V = nullptr;
  const double* xg = nullptr;
  const double* dxs = nullptr;
  double vscale = 1.0, E_mat = 0.0, E_rhs = 0.0, dx = 1.0, dt = 0.0;
  cd* x = nullptr;
  const cd* acc_pa = nullptr;
  const cd* acc_pb = nullptr;
  double* acc_dV = nullptr;
  double* acc_part = nullptr;
  double acc_tau = 0.0;
  int acc_half = 0;
  const double* W = nullptr;  // absorbing potential (SRC_CNW)
  double wscale = 1.0;
  int64_t l0 = 0;  // SRC_LCOUP: partial wave of row 0
};

// Kernel arguments of one launch of a plan for the caller's arrays u and workspace ws.
KArgs plan_args(cn_handle_t h, const Launch& l, const UserArgs& u, char* ws) {
  KArgs a = l.a;
  if (l.level == 1) {
    a.a = u.a;
    a.b = u.b;
    a.c = u.c;
    a.d = u.d;
    a.psi = u.psi;
    a.rhs = u.rhs;
    a.V = u.V;
    a.xg = u.xg;
    a.dxs = u.dxs;
    a.vscale = u.vscale;
    a.E_mat = u.E_mat;
    a.E_rhs = u.E_rhs;
    a.dx = u.dx;
    a.dt = u.dt;
    a.acc_pa = u.acc_pa;
    a.acc_pb = u.acc_pb;
    a.acc_dV = u.acc_dV;
    a.acc_part = u.acc_part;
    a.acc_tau = u.acc_tau;
    a.acc_half = u.acc_half;
    a.Wabs = u.W;
    a.wscale = u.wscale;
    a.l0 = u.l0;
  }
  a.x = (l.o_x >= 0) ? (cd*)(ws + l.o_x) : u.x;
  if (l.o_sU >= 0) a.sU = (const cd*)(ws + l.o_sU);
  if (l.o_sD >= 0) a.sD = (const cd*)(ws + l.o_sD);
  if (l.o_oU >= 0) a.oU = (cd*)(ws + l.o_oU);
  if (l.o_oD >= 0) a.oD = (cd*)(ws + l.o_oD);
  if (l.o_psi_if >= 0) a.psi_if = (const cd*)(ws + l.o_psi_if);
  if (l.o_hout >= 0) a.halo_out = (cd*)(ws + l.o_hout);
  if (l.o_hin >= 0) a.halo_in = (const cd*)(ws + l.o_hin);
  a.status = h->status;
  return a;
}

cn_status launch_k(const void* fn, const Launch& l, KArgs& a, hipStream_t s) {
  void* params[] = {&a};
  if (hipLaunchKernel(fn, l.grid, dim3(l.threads), params, 0, s) != hipSuccess) return CN_ERR_HIP;
  return CN_OK;
}

const char* phase_name(int ph) {
  switch (ph) {
    case nsd::PH_SINGLE: return "single";
    case nsd::PH_REDUCE: return "reduce";
    case nsd::PH_SUBST: return "subst";
    case nsd::PH_FUSE: return "fuse";
  }
  return "persistent";
}

cn_status run_plan(cn_handle_t h, Plan* P, const UserArgs& u, hipStream_t s,
                   void* ws_base = nullptr) {
  char* ws = (char*)(ws_base ? ws_base : h->ws);
  const bool log = h->profiling && !capturing(s);
  for (const Launch& l : P->L) {
    KArgs a = plan_args(h, l, u, ws);
    cn_handle_s::Rec r;
    if (log) {
      char lab[160];
      snprintf(lab, sizeof(lab), "L%d %s %s grid=%ux%u threads=%d", l.level,
               l.fn == aux_fn(nsk::AUX_RS_SERIAL) ? "serial-RS" : phase_name(l.ph),
               l.cfg >= 0 ? cfg_str(l.cfg).c_str() : "-", l.grid.x, l.grid.y, l.threads);
      r.label = lab;
      HIP_TRY(hipEventCreate(&r.e0));
      HIP_TRY(hipEventCreate(&r.e1));
      HIP_TRY(hipEventRecord(r.e0, s));
    }
    cn_status st = launch_k(l.fn, l, a, s);
    if (st != CN_OK) return st;
    if (log) {
      HIP_TRY(hipEventRecord(r.e1, s));
      h->recs.push_back(r);
    }
  }
  return CN_OK;
}

// Cross-step fusion of a Crank-Nicolson sequence (Sec. 5.3 fuses the explicit half-step into
// the solve; here the solve's second pass also takes the next step's first pass).  A plan
// qualifies when its level-1 launches are whole-system tiles plus one two-pass group (first
// pass, the levels of its reduced system, second pass) of row tiles.
struct FusePlan {
  bool ok = false;
  int red = -1, sub = -1;
  std::vector<int> singles, mids;
  // the fused pass's last workgroup solves the reduced system (one system whose tile joints
  // fit one whole-system tile of 2 rows per lane of the pass's workgroup): no launch of its own
  bool inl = false;
};

// reduced systems of fused passes solved inside the pass (CN_INLINE=0 turns it off: a launch
// of their own after every pass)
bool inline_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_INLINE");
    return !(e && e[0] == '0');
  }();
  return on;
}

FusePlan fuse_plan(const Plan* P) {
  FusePlan f;
  for (int i = 0; i < (int)P->L.size(); ++i) {
    const Launch& l = P->L[i];
    if (l.level == 1) {
      if (l.cfg < 0 || !nsd::cn_src(l.src) || !g_kern[l.cfg][l.src][nsd::PH_FUSE]) return f;
      if (l.ph == nsd::PH_SINGLE && l.fn == g_kern[l.cfg][l.src][nsd::PH_SINGLE] && f.red < 0) {
        f.singles.push_back(i);
      } else if (l.ph == nsd::PH_REDUCE && f.red < 0 && l.o_hout2 >= 0 &&
                 l.fn == g_kern[l.cfg][l.src][nsd::PH_REDUCE]) {
        f.red = i;
      } else if (l.ph == nsd::PH_SUBST && f.red >= 0 && f.sub < 0 &&
                 l.fn == g_kern[l.cfg][l.src][nsd::PH_SUBST] && l.cfg == P->L[f.red].cfg) {
        f.sub = i;
      } else {
        return f;
      }
    } else {
      if (f.red < 0 || f.sub >= 0) return f;
      f.mids.push_back(i);
    }
  }
  f.ok = f.red >= 0 && f.sub >= 0;
  if (f.ok && f.mids.size() == 1 && inline_enabled()) {
    const Launch& R = P->L[f.red];
    const Launch& S = P->L[f.sub];
    const Launch& m = P->L[f.mids[0]];
    // level 1: one system of a uniform layout in K tiles; level 2: its reduced system of K rows
    // as one whole-system tile, reading the first pass's slots and writing where the second
    // pass reads.  Taken when that tile of 2 rows per lane is more than half full (64 W < K <=
    // 128 W): measured on 2^16 .. 2^20-row chains, a fuller in-pass solve saves the launch
    // (2^20 rows in 512 tiles of 8 rows per lane, with a field: forward 55.2 -> 53.1 ms and
    // reverse mode 88.2 -> 81.4 ms over 2000 steps), an emptier one costs more than the
    // launch it saves (every workgroup then waits for its stores and its count to return).
    const int64_t Wp = kCfgs[S.cfg].W;
    f.inl = S.t_wgs < 0 && S.grid.y == 1 && R.grid.y == 1 && S.a.ntiles > 64 * Wp &&
            S.a.ntiles <= 128 * Wp && m.level == 2 &&
            m.src == nsd::SRC_SLOTS && m.ph == nsd::PH_SINGLE && m.cfg >= 0 &&
            m.fn == g_kern[m.cfg][nsd::SRC_SLOTS][nsd::PH_SINGLE] && m.grid.x == 1 &&
            m.grid.y == 1 && m.o_x >= 0 && m.o_x == S.o_psi_if && m.o_sU == R.o_oU &&
            m.o_sD == R.o_oD;
  }
  return f;
}

// cross-step fusion of cn_propagate (CN_FUSE=0 turns it off)
bool fuse_enabled() {
  static const bool on = [] {
    const char* e = getenv("CN_FUSE");
    return !(e && e[0] == '0');
  }();
  return on;
}

// A chain of nst >= 1 Crank-Nicolson steps over a plan with one fusable two-pass group.
// args(i) gives step i's arrays, field (E_mat = E_rhs) and accumulation; before(i) runs before
// step i writes its new state, after(i) once it has.  Launches: first pass of step 0; the
// levels above; then per step i: whole-system tiles, and either PH_FUSE (second pass of step i
// + first pass of step i+1; the levels above then add the deferred joint-row terms from its
// edge rows) or, at the last step, the second pass.  The two edge-row arrays alternate: a pass
// reads the state's edge rows written by the pass before and writes those of its own new
// state.  Second passes of large levels alternate their direction, so that each starts on the
// tiles its predecessor wrote last.
using StepArgs = std::function<UserArgs(int64_t)>;
using StepHook = std::function<cn_status(int64_t)>;

cn_status run_chain(cn_handle_t h, Plan* P, const FusePlan& f, int64_t nst, const StepArgs& args,
                    const StepHook& before, const StepHook& after, hipStream_t s,
                    void* ws_base = nullptr) {
  char* ws = (char*)(ws_base ? ws_base : h->ws);
  const Launch& R = P->L[f.red];
  const Launch& S = P->L[f.sub];
  cd* H[2] = {(cd*)(ws + R.o_hout), (cd*)(ws + R.o_hout2)};
  // the done count of an inline reduced solve: one per workspace, since chains on the two
  // workspaces may run at once on two streams
  int* inl = nullptr;
  if (f.inl) {
    if (ws == (char*)h->ws) inl = h->sync;
    else if (ws == (char*)h->ws2) inl = h->sync + 32;
  }
  auto mids = [&](const cd* hal, const UserArgs& u) -> cn_status {
    for (int i : f.mids) {
      const Launch& l = P->L[i];
      KArgs a = plan_args(h, l, u, ws);
      if (hal && l.level == 2) {
        a.ud_halo = hal;
        a.dt = u.dt;
        a.dx = u.dx;
        a.dxs = u.dxs;
      }
      cn_status st = launch_k(l.fn, l, a, s);
      if (st != CN_OK) return st;
    }
    return CN_OK;
  };
  cn_status st;
  UserArgs v = args(0);
  {
    KArgs a = plan_args(h, R, v, ws);
    a.halo_out = H[0];
    if ((st = launch_k(R.fn, R, a, s)) != CN_OK) return st;
  }
  if ((st = mids(nullptr, v)) != CN_OK) return st;
  for (int64_t i = 0; i < nst; ++i) {
    if (before && (st = before(i)) != CN_OK) return st;
    for (int l : f.singles) {
      KArgs a = plan_args(h, P->L[l], v, ws);
      if ((st = launch_k(P->L[l].fn, P->L[l], a, s)) != CN_OK) return st;
    }
    KArgs a = plan_args(h, S, v, ws);
    a.halo_in = H[i & 1];
    a.rev = S.a.rev ? (int)((i & 1) == 0) : 0;
    if (i + 1 < nst) {
      const UserArgs vn = args(i + 1);
      a.halo_out = H[(i + 1) & 1];
      a.oU = (cd*)(ws + R.o_oU);
      a.oD = (cd*)(ws + R.o_oD);
      a.E_next = vn.E_mat;
      a.inl_sync = inl;
      if ((st = launch_k(g_kern[S.cfg][S.src][nsd::PH_FUSE], S, a, s)) != CN_OK) return st;
      if (after && (st = after(i)) != CN_OK) return st;
      if (!inl && (st = mids(H[(i + 1) & 1], vn)) != CN_OK) return st;
      v = vn;
    } else {
      if ((st = launch_k(S.fn, S, a, s)) != CN_OK) return st;
      if (after && (st = after(i)) != CN_OK) return st;
    }
  }
  return CN_OK;
}

nsd::AuxArgs aux_from(const cn_layout* L, const Plan* P) {
  nsd::AuxArgs x{};
  x.n = L->n;
  x.batch = L->batch;
  x.es = L->elem_stride;
  x.bs = L->batch_stride;
  x.total = P->rows;
  x.vscale = 1.0;
  x.wscale = 1.0;
  return x;
}

int64_t* dev_offsets(const Plan* P) {
  // the first uneven launch at level 1 carries the caller's offsets table
  for (const Launch& l : P->L)
    if (l.level == 1 && l.a.offs) return const_cast<int64_t*>(l.a.offs);
  return nullptr;
}

cn_status launch_aux(const void* fn, int64_t rows, nsd::AuxArgs& x, hipStream_t s) {
  const unsigned blocks = (unsigned)((rows + 255) / 256);
  void* params[] = {&x};
  if (hipLaunchKernel(fn, dim3(blocks), dim3(256), params, 0, s) != hipSuccess) return CN_ERR_HIP;
  return CN_OK;
}

// out[r] = sum of row r of part (rows of nparts values), r < rows, in a fixed order
cn_status launch_sum_partials(const double* part, int64_t nparts, double* out, int64_t rows,
                              hipStream_t s) {
  void* params[] = {&part, &nparts, &out};
  if (hipLaunchKernel(aux_fn(nsk::AUX_SUM_PARTIALS), dim3((unsigned)rows), dim3(256), params, 0,
                      s) != hipSuccess)
    return CN_ERR_HIP;
  return CN_OK;
}

cn_status check_op(const cn_operator* op) {
  if (!op || !op->V) return CN_ERR_INVALID_ARG;
  if (!op->dx_per_system && !(op->dx > 0.0)) return CN_ERR_INVALID_ARG;
  if (!(op->dt == op->dt)) return CN_ERR_INVALID_ARG;
  return CN_OK;
}

nsd::AuxArgs aux_op(const cn_layout* L, const Plan* P, const cn_operator* op, double E) {
  nsd::AuxArgs X = aux_from(L, P);
  X.offs = dev_offsets(P);
  X.V = op->V;
  X.xg = op->xgrid;
  X.vscale = op->v_scale;
  X.E = E;
  X.dx = op->dx;
  X.dxs = op->dx_per_system;
  X.dt = op->dt;
  X.W = op->absorb;
  return X;
}

// A Crank-Nicolson step whose potential has an absorbing part (V - iW): T and the explicit
// side 1 - i tau H are no longer each other's adjoints and T's diagonal has a real part other
// than 1, so the step is taken in materialised form -- a, b, c and d = (1 - i tau H) psi_in in
// the handle's buffer, then the general solve of the same layout.  coeffs = false reuses a, b, c
// from the previous call (same operator and field).
cn_status absorbing_step(cn_handle_t h, const cn_layout* L, const cn_operator* op, double E,
                         bool coeffs, const cd* psi_in, cd* psi_out, hipStream_t s) {
  if (L && L->shared_coefficients == 1) return CN_ERR_UNSUPPORTED;
  Plan* P = nullptr;
  cn_status st = get_plan(h, L, nsd::SRC_CN, s, &P);
  if (st != CN_OK) return st;
  Plan* Pe = nullptr;
  st = get_plan(h, L, nsd::SRC_EXPL, s, &Pe);
  if (st != CN_OK) return st;
  const int64_t sp = P->span;
  const size_t need = 4 * (size_t)sp * sizeof(cd);
  if (h->mat_size < need) {
    if (capturing(s)) return CN_ERR_NOT_RESERVED;
    st = regrow(h, &h->mat, &h->mat_size, need);
    if (st != CN_OK) return st;
    coeffs = true;
  }
  cd* m = (cd*)h->mat;
  nsd::AuxArgs X = aux_op(L, P, op, E);
  if (coeffs) {
    X.a = m;
    X.b = m + sp;
    X.c = m + 2 * sp;
    st = launch_aux(aux_fn(nsk::AUX_ASSEMBLE), P->rows, X, s);
    if (st != CN_OK) return st;
  }
  X.psi = psi_in;
  X.d = m + 3 * sp;
  st = launch_aux(aux_fn(nsk::AUX_RHS), P->rows, X, s);
  if (st != CN_OK) return st;
  UserArgs u;
  u.a = m;
  u.b = m + sp;
  u.c = m + 2 * sp;
  u.d = m + 3 * sp;
  u.x = psi_out;
  return run_plan(h, Pe, u, s);
}

// The plan of a Crank-Nicolson step for this operator: SRC_CN for real potentials, SRC_CNW (the
// fused kernels with the absorbing term) when the potential has one.  *fused is false when an
// absorbing step has to run materialised instead (fused kernels turned off, or a layout whose
// configuration they are not built for); P is then null.
cn_status cn_plan(cn_handle_t h, const cn_layout* L, const cn_operator* op, hipStream_t s,
                  Plan** P, bool* fused) {
  *P = nullptr;
  *fused = true;
  if (!op->absorb) return get_plan(h, L, nsd::SRC_CN, s, P);
  if (L && L->shared_coefficients == 1) return CN_ERR_UNSUPPORTED;
  if (absorb_fused_enabled()) {
    const cn_status st = get_plan(h, L, nsd::SRC_CNW, s, P);
    if (st != CN_ERR_UNSUPPORTED) return st;
    *P = nullptr;
  }
  *fused = false;
  return CN_OK;
}

// Step arguments of a Crank-Nicolson operator (state in, state out, field E on both sides).
UserArgs cn_args(const cn_operator* op, double E, const cd* in, cd* out) {
  UserArgs u;
  u.psi = in;
  u.V = op->V;
  u.xg = op->xgrid;
  u.dxs = op->dx_per_system;
  u.vscale = op->v_scale;
  u.E_mat = E;
  u.E_rhs = E;
  u.dx = op->dx;
  u.dt = op->dt;
  u.x = out;
  u.W = op->absorb;
  u.wscale = 1.0;
  return u;
}

}  // namespace

// =============================================================================== C ABI
extern "C" {

const char* cn_version(void) { return "cntri 0.1 (gfx950, FP64, N-shaped partition method)"; }

const char* cn_status_string(cn_status st) {
  switch (st) {
    case CN_OK: return "CN_OK";
    case CN_NUMERICAL_BREAKDOWN: return "CN_NUMERICAL_BREAKDOWN";
    case CN_ERR_INVALID_ARG: return "CN_ERR_INVALID_ARG";
    case CN_ERR_UNSUPPORTED: return "CN_ERR_UNSUPPORTED";
    case CN_ERR_NO_MEMORY: return "CN_ERR_NO_MEMORY";
    case CN_ERR_HIP: return "CN_ERR_HIP";
    case CN_ERR_NOT_RESERVED: return "CN_ERR_NOT_RESERVED";
    case CN_ERR_SCRATCH_TOO_SMALL: return "CN_ERR_SCRATCH_TOO_SMALL";
    case CN_ERR_WAIT_TIMEOUT: return "CN_ERR_WAIT_TIMEOUT";
  }
  return "unknown cn_status";
}

cn_status cn_check_layout(const cn_layout* layout) {
  int64_t rows = 0, span = 0;
  return validate(layout, rows, span);
}

cn_status cn_create(cn_handle_t* handle, int device) {
  if (!handle) return CN_ERR_INVALID_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return CN_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return CN_ERR_HIP;
  cn_handle_s* h = new cn_handle_s();
  h->device = device;
  if (hipMalloc(&h->status, 128 * sizeof(int)) != hipSuccess) {
    delete h;
    return CN_ERR_NO_MEMORY;
  }
  h->sync = h->status + 64;
  if (hipMemset(h->status, 0, 128 * sizeof(int)) != hipSuccess ||
      scratch_setup(device, &h->scratch) != CN_OK) {
    (void)hipFree(h->status);
    delete h;
    return CN_ERR_HIP;
  }
  *handle = h;
  return CN_OK;
}

cn_status cn_destroy(cn_handle_t h) {
  if (!h) return CN_ERR_INVALID_ARG;
  (void)hipDeviceSynchronize();
  h->plans.clear();
  h->static_plans.clear();
  if (h->ws) (void)hipFree(h->ws);
  if (h->rows_buf) (void)hipFree(h->rows_buf);
  if (h->ws2) (void)hipFree(h->ws2);
  if (h->seg2) (void)hipFree(h->seg2);
  if (h->mat) (void)hipFree(h->mat);
  if (h->rad) (void)hipFree(h->rad);
  if (h->res) (void)hipFree(h->res);
  for (void* p : h->retired) (void)hipFree(p);
  for (auto& r : h->recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  for (hipEvent_t e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  if (h->status) (void)hipFree(h->status);
  delete h;
  return CN_OK;
}

namespace {
cn_status reserve_resident(cn_handle_t h, const cn_layout* L);
}

cn_status cn_reserve(cn_handle_t h, const cn_layout* L) {
  if (!h) return CN_ERR_INVALID_ARG;
  {
    const cn_status st = reserve_resident(h, L);
    if (st != CN_OK) return st;
  }
  Plan* P = nullptr;
  size_t ws2 = 0;  // the second workspace of the reverse mode's fused chain
  for (int src : {nsd::SRC_EXPL, nsd::SRC_EXPL_CT, nsd::SRC_CN, nsd::SRC_CNW, nsd::SRC_LCOUP}) {
    cn_status st = get_plan(h, L, src, nullptr, &P);
    if (st == CN_ERR_UNSUPPORTED && (src == nsd::SRC_CNW || src == nsd::SRC_LCOUP)) continue;
    if (st != CN_OK) return st;
    if (nsd::cn_src(src)) ws2 = std::max(ws2, P->ws_bytes);
  }
  if (h->ws2_size < ws2) return regrow(h, &h->ws2, &h->ws2_size, ws2);
  return CN_OK;
}

cn_status cn_describe_plan(cn_handle_t h, const cn_layout* L, int cn_mode, char* buf,
                           int64_t buflen) {
  if (!h || !buf || buflen < 1 || cn_mode < 0 || cn_mode > 2) return CN_ERR_INVALID_ARG;
  Plan* P = nullptr;
  const int src = cn_mode == 2 ? nsd::SRC_CNW : cn_mode ? nsd::SRC_CN : nsd::SRC_EXPL;
  cn_status st = get_plan(h, L, src, nullptr, &P);
  if (st != CN_OK) return st;
  std::string d = P->desc;
  if (cn_mode) {
    // how cn_propagate runs this plan
    const FusePlan f = fuse_enabled() ? fuse_plan(P) : FusePlan();
    if (f.ok)
      d += f.inl ? "chain: one fused pass per step, reduced system solved in the pass; "
                 : "chain: one fused pass per step; ";
  }
  snprintf(buf, (size_t)buflen, "%s", d.c_str());
  return CN_OK;
}

cn_status cn_tridiag_solve(cn_handle_t h, const cn_layout* L, const void* a, const void* b,
                           const void* c, const void* d, void* x, cn_stream_t stream) {
  if (!h || !a || !b || !c || !d || !x) return CN_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  Plan* P = nullptr;
  cn_status st = get_plan(h, L, nsd::SRC_EXPL, s, &P);
  if (st != CN_OK) return st;
  UserArgs u;
  u.a = (const cd*)a;
  u.b = (const cd*)b;
  u.c = (const cd*)c;
  u.d = (const cd*)d;
  u.x = (cd*)x;
  return run_plan(h, P, u, s);
}

cn_status cn_tridiag_solve_noalloc(cn_handle_t h, const cn_layout* L, const void* a,
                                   const void* b, const void* c, const void* d, void* x,
                                   cn_stream_t stream) {
  if (!h || !a || !b || !c || !d || !x) return CN_ERR_INVALID_ARG;
  if (!h->scratch) return CN_ERR_HIP;
  int64_t rows = 0, span = 0;
  cn_status st = validate(L, rows, span);
  if (st != CN_OK) return st;
  // the plan of this layout, built on the host on the first call (no device memory); its
  // tables are bound to the start of the scratch array and its workspace follows them
  const std::string key = plan_key(L, nsd::SRC_EXPL);
  auto it = h->static_plans.find(key);
  if (it == h->static_plans.end()) {
    std::unique_ptr<Plan> P(new Plan());
    std::vector<char> tab;
    st = build_plan(L, nsd::SRC_EXPL, false, *P, tab);
    if (st != CN_OK) return st;
    P->host_tab.swap(tab);
    bind_tables(*P, h->scratch);
    it = h->static_plans.emplace(key, std::move(P)).first;
  }
  Plan* P = it->second.get();
  const size_t tab_bytes = (P->host_tab.size() + 255) & ~size_t(255);
  if (tab_bytes + P->ws_bytes > kScratchBytes) return CN_ERR_SCRATCH_TOO_SMALL;
  hipStream_t s = (hipStream_t)stream;
  // the tables are copied on every call: another call may have used the array since
  if (!P->host_tab.empty() &&
      hipMemcpyAsync(h->scratch, P->host_tab.data(), P->host_tab.size(), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return CN_ERR_HIP;
  UserArgs u;
  u.a = (const cd*)a;
  u.b = (const cd*)b;
  u.c = (const cd*)c;
  u.d = (const cd*)d;
  u.x = (cd*)x;
  return run_plan(h, P, u, s, h->scratch + tab_bytes);
}

cn_status cn_tridiag_solve_adjoint(cn_handle_t h, const cn_layout* L, const void* a,
                                   const void* b, const void* c, const void* x, const void* gx,
                                   void* gd, void* ga, void* gb, void* gc, cn_stream_t stream) {
  if (!h || !a || !b || !c || !x || !gx || !gd) return CN_ERR_INVALID_ARG;
  if (L && L->shared_coefficients == 1) return CN_ERR_UNSUPPORTED;
  if (gd == x || gd == a || gd == b || gd == c) return CN_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  Plan* P = nullptr;
  cn_status st = get_plan(h, L, nsd::SRC_EXPL_CT, s, &P);
  if (st != CN_OK) return st;
  UserArgs u;
  u.a = (const cd*)a;
  u.b = (const cd*)b;
  u.c = (const cd*)c;
  u.d = (const cd*)gx;
  u.x = (cd*)gd;
  st = run_plan(h, P, u, s);
  if (st != CN_OK) return st;
  if (ga || gb || gc) {
    nsd::AuxArgs X = aux_from(L, P);
    X.offs = dev_offsets(P);
    X.lam = (const cd*)gd;
    X.xsol = (const cd*)x;
    X.ga = (cd*)ga;
    X.gb = (cd*)gb;
    X.gc = (cd*)gc;
    st = launch_aux(aux_fn(nsk::AUX_SOLVE_GRADS), P->rows, X, s);
  }
  return st;
}

cn_status cn_assemble(cn_handle_t h, const cn_layout* L, const cn_operator* op, double E, void* a,
                      void* b, void* c, cn_stream_t stream) {
  if (!h || !a || !b || !c) return CN_ERR_INVALID_ARG;
  if (L && L->shared_coefficients == 1) return CN_ERR_UNSUPPORTED;
  cn_status st = check_op(op);
  if (st != CN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Plan* P = nullptr;
  st = get_plan(h, L, nsd::SRC_CN, s, &P);
  if (st != CN_OK) return st;
  nsd::AuxArgs X = aux_op(L, P, op, E);
  X.a = (cd*)a;
  X.b = (cd*)b;
  X.c = (cd*)c;
  return launch_aux(aux_fn(nsk::AUX_ASSEMBLE), P->rows, X, s);
}

cn_status cn_rhs(cn_handle_t h, const cn_layout* L, const cn_operator* op, double E,
                 const void* psi, void* d, cn_stream_t stream) {
  if (!h || !psi || !d || psi == d) return CN_ERR_INVALID_ARG;
  if (L && L->shared_coefficients == 1) return CN_ERR_UNSUPPORTED;
  cn_status st = check_op(op);
  if (st != CN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Plan* P = nullptr;
  st = get_plan(h, L, nsd::SRC_CN, s, &P);
  if (st != CN_OK) return st;
  nsd::AuxArgs X = aux_op(L, P, op, E);
  X.psi = (const cd*)psi;
  X.d = (cd*)d;
  return launch_aux(aux_fn(nsk::AUX_RHS), P->rows, X, s);
}

cn_status cn_step(cn_handle_t h, const cn_layout* L, const cn_operator* op, double E,
                  const void* psi_in, void* psi_out, cn_stream_t stream) {
  if (!h || !psi_in || !psi_out) return CN_ERR_INVALID_ARG;
  cn_status st = check_op(op);
  if (st != CN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Plan* P = nullptr;
  bool fused = true;
  st = cn_plan(h, L, op, s, &P, &fused);
  if (st != CN_OK) return st;
  if (!fused) return absorbing_step(h, L, op, E, true, (const cd*)psi_in, (cd*)psi_out, s);
  return run_plan(h, P, cn_args(op, E, (const cd*)psi_in, (cd*)psi_out), s);
}

cn_status cn_propagate(cn_handle_t h, const cn_layout* L, const cn_operator* op, int64_t nsteps,
                       const double* E, void* psi, void* ckpt, int64_t K, cn_stream_t stream) {
  if (!h || !psi || nsteps < 0) return CN_ERR_INVALID_ARG;
  if (ckpt && K < 1) return CN_ERR_INVALID_ARG;
  cn_status st = check_op(op);
  if (st != CN_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Plan* P = nullptr;
  bool fused = true;
  st = cn_plan(h, L, op, s, &P, &fused);
  if (st != CN_OK) return st;
  if (!fused) {
    st = get_plan(h, L, nsd::SRC_CN, s, &P);
    if (st != CN_OK) return st;
    for (int64_t k = 0; k < nsteps; ++k) {
      if (ckpt && k % K == 0)
        HIP_TRY(hipMemcpyAsync((cd*)ckpt + (k / K) * P->span, psi, P->span * sizeof(cd),
                               hipMemcpyDeviceToDevice, s));
      // without a field T is the same every step: assemble it once
      st = absorbing_step(h, L, op, E ? E[k] : 0.0, k == 0 || E != nullptr, (const cd*)psi,
                          (cd*)psi, s);
      if (st != CN_OK) return st;
    }
    return CN_OK;
  }
  UserArgs u = cn_args(op, 0.0, (const cd*)psi, (cd*)psi);
  if (nsteps >= 2 && fuse_enabled()) {
    const FusePlan f = fuse_plan(P);
    if (f.ok) {
      auto args = [&](int64_t k) {
        UserArgs v = u;
        v.E_mat = v.E_rhs = E ? E[k] : 0.0;
        return v;
      };
      auto before = [&](int64_t k) -> cn_status {
        if (ckpt && k % K == 0)
          HIP_TRY(hipMemcpyAsync((cd*)ckpt + (k / K) * P->span, psi, P->span * sizeof(cd),
                                 hipMemcpyDeviceToDevice, s));
        return CN_OK;
      };
      return run_chain(h, P, f, nsteps, args, before, nullptr, s);
    }
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    if (ckpt && k % K == 0) {
      HIP_TRY(hipMemcpyAsync((cd*)ckpt + (k / K) * P->span, psi, P->span * sizeof(cd),
                             hipMemcpyDeviceToDevice, s));
    }
    u.E_mat = u.E_rhs = E ? E[k] : 0.0;
    st = run_plan(h, P, u, s);
    if (st != CN_OK) return st;
  }
  return CN_OK;
}

// Resident propagation (k_resident): the configuration for n rows, or -1.  The smallest tile
// whose count K is at most 128 (the reduced solve of one wavefront), else the smallest whose K
// fits the reduced solve of its workgroup (128 W joints); always K within the GPU at once.
// Measured per step, no field: 2^18 rows 11.8 us with 2048-row tiles (K = 128) against 13.0 us
// with 1024-row tiles (K = 256); 65536 rows 9.6 us with 512-row tiles against 9.9 and 10.9.
namespace {
bool resident_enabled() {
  const char* e = getenv("CN_RESIDENT");
  return !(e && e[0] == '0');
}
int resident_spin() {
  const char* e = getenv("CN_RESIDENT_SPIN");  // polls before a wait gives up (tests)
  if (e && *e) {
    const long v = strtol(e, nullptr, 10);
    if (v >= 0 && v <= INT_MAX) return (int)v;
  }
  return 1 << 22;
}
// wa: the kernel for a potential with an absorbing part
int64_t resident_capacity(int ci, int wa) {
  static std::mutex mu;
  static int64_t cap[nsk::kNumResCfg][2] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (cap[ci][wa] == 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, nsk::tables().res[ci][wa],
                                                     64 * nsk::kResCfgs[ci].W, 0) != hipSuccess ||
        per_cu < 1) {
      (void)hipGetLastError();
      per_cu = 0;
    }
    cap[ci][wa] = per_cu > 0 ? (int64_t)per_cu * num_cus() : -1;
  }
  return cap[ci][wa];
}
int resident_cfg(int64_t n, int64_t partition, int wa) {
  for (const int64_t lim : {(int64_t)128, (int64_t)0}) {
    for (int ci = 0; ci < nsk::kNumResCfg; ++ci) {
      const Cfg c = nsk::kResCfgs[ci];
      if (partition > 0 && c.T() != partition) continue;
      const int64_t K = (n + c.T() - 1) / c.T();
      if (K <= (lim ? lim : 128 * c.W) && K <= resident_capacity(ci, wa)) return ci;
    }
  }
  return -1;
}
// Bytes of the resident propagation's buffer for K tiles (and nsteps field values): a flag per
// tile (a fixed area for the most tiles any configuration takes, zero between launches), then
// two parity buffers each of slots (3 + 3 per tile) and edge rows (2 per tile), then the field.
constexpr int64_t kResMaxTiles = 128 * 4;
struct ResLayout {
  size_t o_oU, o_oD, o_h, o_E;
  ResLayout(int64_t K)
      : o_oU(kResMaxTiles * sizeof(int)),
        o_oD(o_oU + 6 * K * sizeof(cd)),
        o_h(o_oD + 6 * K * sizeof(cd)),
        o_E(o_h + 4 * K * sizeof(cd)) {}
};

// A layout the resident propagation takes (either potential kind), and its tile configuration.
bool resident_layout(const cn_layout* L, int wa, int* ci) {
  int64_t rows = 0, span = 0;
  if (validate(L, rows, span) != CN_OK) return false;
  if (!resident_enabled() || L->offsets || L->batch != 1 || L->elem_stride != 1 ||
      L->shared_coefficients || L->levels || (L->rows_per_thread && L->rows_per_thread != 8))
    return false;
  *ci = resident_cfg(L->n, L->partition, wa);
  return *ci >= 0;
}

cn_status grow_resident(cn_handle_t h, size_t need) {
  if (need <= h->res_size) return CN_OK;
  const cn_status st = regrow(h, &h->res, &h->res_size, need);
  if (st != CN_OK) return st;
  HIP_TRY(hipMemset(h->res, 0, need));  // the flags start at zero (never inside a capture)
  return CN_OK;
}

// cn_reserve: the buffer of a resident propagation without a field on this layout
cn_status reserve_resident(cn_handle_t h, const cn_layout* L) {
  for (int wa = 0; wa < 2; ++wa) {
    int ci = -1;
    if (!resident_layout(L, wa, &ci)) continue;
    const int64_t T = nsk::kResCfgs[ci].T(), K = (L->n + T - 1) / T;
    const cn_status st = grow_resident(h, ResLayout(K).o_E);
    if (st != CN_OK) return st;
  }
  return CN_OK;
}
}  // namespace

cn_status cn_propagate_resident(cn_handle_t h, const cn_layout* L, const cn_operator* op,
                                int64_t nsteps, const double* E, void* psi, void* ckpt,
                                int64_t K_ckpt, cn_stream_t stream) {
  if (!h || !psi || nsteps < 0 || nsteps > INT_MAX - 2) return CN_ERR_INVALID_ARG;
  if (ckpt && (K_ckpt < 1 || K_ckpt > INT_MAX)) return CN_ERR_INVALID_ARG;
  cn_status st = check_op(op);
  if (st != CN_OK) return st;
  int64_t rows = 0, span = 0;
  st = validate(L, rows, span);
  if (st != CN_OK) return st;
  const int wa = op->absorb ? 1 : 0;
  int ci = -1;
  if (op->dx_per_system || !resident_layout(L, wa, &ci)) return CN_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  const bool cap = capturing(s);
  if (E && cap) return CN_ERR_UNSUPPORTED;  // the field is uploaded by a host copy
  if (nsteps == 0) return CN_OK;
  const int64_t T = nsk::kResCfgs[ci].T(), K = (L->n + T - 1) / T;
  const ResLayout RL(K);
  const size_t o_oU = RL.o_oU, o_oD = RL.o_oD, o_h = RL.o_h, o_E = RL.o_E;
  const size_t need = o_E + (E ? (size_t)nsteps * sizeof(double) : 0);
  if (cap) h->captured = true;
  if (need > h->res_size) {
    if (cap) return CN_ERR_NOT_RESERVED;
    st = grow_resident(h, need);
    if (st != CN_OK) return st;
  }
  char* w = (char*)h->res;
  if (E) HIP_TRY(hipMemcpyAsync(w + o_E, E, nsteps * sizeof(double), hipMemcpyHostToDevice, s));
  if (ckpt)  // the state before step 0
    HIP_TRY(hipMemcpyAsync(ckpt, psi, L->n * sizeof(cd), hipMemcpyDeviceToDevice, s));
  KArgs a{};
  a.n = L->n;
  a.ntiles = K;
  a.es = 1;
  a.bs = L->n;
  a.psi = (const cd*)psi;
  a.x = (cd*)psi;
  a.V = op->V;
  a.xg = op->xgrid;
  a.vscale = op->v_scale;
  a.dx = op->dx;
  a.dt = op->dt;
  a.Wabs = op->absorb;
  a.wscale = 1.0;
  a.oU = (cd*)(w + o_oU);
  a.oD = (cd*)(w + o_oD);
  a.halo_out = (cd*)(w + o_h);
  a.status = h->status;
  nsd::ResArgs r{};
  r.E = E ? (const double*)(w + o_E) : nullptr;
  r.nsteps = (int)nsteps;
  r.flags = (int*)w;
  r.sync = h->status + 96;
  r.spin = resident_spin();
  r.bufstep = K;
  r.ckpt = (cd*)ckpt;
  r.K = ckpt ? (int)K_ckpt : 1;
  void* params[] = {&a, &r};
  if (hipLaunchKernel(nsk::tables().res[ci][wa], dim3((unsigned)K),
                      dim3(64 * nsk::kResCfgs[ci].W),
                      params, 0, s) != hipSuccess)
    return CN_ERR_HIP;
  return CN_OK;
}

cn_status cn_step_adjoint(cn_handle_t h, const cn_layout* L, const cn_operator* op, double E,
                          const void* psi_n, const void* psi_np1, const void* g_np1, void* g_n,
                          double* dV_accum, double* dE_partial, cn_stream_t stream) {
  if (!h || !psi_n || !psi_np1 || !g_np1 || !g_n) return CN_ERR_INVALID_ARG;
  if (L && L->shared_coefficients == 1) return CN_ERR_UNSUPPORTED;
  cn_status st = check_op(op);
  if (st != CN_OK) return st;
  if (dE_partial && !op->xgrid) return CN_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  Plan* P = nullptr;
  bool fused = true;
  st = cn_plan(h, L, op, s, &P, &fused);
  if (st != CN_OK) return st;
  if (!fused) return CN_ERR_UNSUPPORTED;
  cd* lam = (cd*)((char*)h->ws + P->o_aux);
  // lambda = T^{-H} g: T^H = 1 + tau W - i tau (...) is the CN matrix with dt -> -dt and
  // W -> -W (for a real potential simply dt -> -dt)
  UserArgs u = cn_args(op, E, (const cd*)g_np1, lam);
  u.rhs = (const cd*)g_np1;
  u.dt = -op->dt;
  u.wscale = -1.0;
  st = run_plan(h, P, u, s);
  if (st != CN_OK) return st;
  // g_n = B^H lambda with B = 1 - i tau H: the explicit half-step with dt -> -dt and W -> -W
  // (for a real potential B^H = T = 1 + i tau H)
  nsd::AuxArgs X = aux_from(L, P);
  X.offs = dev_offsets(P);
  X.V = op->V;
  X.xg = op->xgrid;
  X.vscale = op->v_scale;
  X.E = E;
  X.dx = op->dx;
  X.dxs = op->dx_per_system;
  X.dt = -op->dt;
  X.W = op->absorb;
  X.wscale = -1.0;
  X.psi = lam;
  X.d = (cd*)g_n;
  st = launch_aux(aux_fn(nsk::AUX_RHS), P->rows, X, s);
  if (st != CN_OK) return st;
  // gradient terms
  nsd::AuxArgs Y = aux_from(L, P);
  Y.offs = X.offs;
  Y.xg = op->xgrid;
  Y.vscale = op->v_scale;
  Y.dt = op->dt;
  Y.lam = lam;
  Y.psi_n = (const cd*)psi_n;
  Y.psi_np1 = (const cd*)psi_np1;
  Y.dV = dV_accum;
  double* part = (double*)((char*)h->ws + P->o_part);
  Y.dE_part = dE_partial ? part : nullptr;
  st = launch_aux(aux_fn(nsk::AUX_ADJ_ACCUM), P->rows, Y, s);
  if (st != CN_OK) return st;
  if (dE_partial) {
    st = launch_sum_partials(part, (int64_t)((P->rows + 255) / 256), dE_partial, 1, s);
    if (st != CN_OK) return st;
  }
  return CN_OK;
}

cn_status cn_autotune(cn_handle_t h, const cn_layout* L, int cn_mode, const cn_operator* op,
                      double E, const void* a, const void* b, const void* c, const void* d,
                      void* x, char* report, int64_t report_len, cn_stream_t stream) {
  if (!h || !L || !d || !x || d == x) return CN_ERR_INVALID_ARG;
  if (cn_mode && check_op(op) != CN_OK) return CN_ERR_INVALID_ARG;
  if (cn_mode && op->absorb) return CN_ERR_UNSUPPORTED;
  if (!cn_mode && (!a || !b || !c)) return CN_ERR_INVALID_ARG;
  if (L->partition != 0 || L->rows_per_thread != 0) return CN_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (capturing(s)) return CN_ERR_NOT_RESERVED;
  const int src = cn_mode ? nsd::SRC_CN : nsd::SRC_EXPL;
  const int64_t kSeq = 8;  // cn_mode 2: steps of the timed sequence
  int64_t span = 0;
  {
    int64_t rows = 0;
    if (validate(L, rows, span) != CN_OK) return CN_ERR_INVALID_ARG;
  }
  struct Cand {
    int T, M;
  };
  std::vector<Cand> cands = {{0, 0},    {128, 2},  {256, 4},  {512, 4},  {1024, 4}, {2048, 4},
                             {4096, 4}, {512, 8},  {1024, 8}, {2048, 8}, {4096, 8}};
  // interleaved batches run the column kernels: their tiles of T = W M rows are the candidates
  if (!L->offsets && L->batch_stride == 1 && L->batch >= 64 && L->elem_stride >= L->batch &&
      !L->shared_coefficients) {
    cands.resize(1);
    for (const Cfg& c : kColCfgs) cands.push_back({c.M * c.W, c.M});
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::string rep;
  float best = 1e30f;
  std::string best_key;
  int best_T = 0, best_M = 0;
  for (const Cand& cd_ : cands) {
    cn_layout L2 = *L;
    L2.partition = cd_.T;
    L2.rows_per_thread = cd_.M;
    if (L->offsets && cd_.T > 0) {  // persistent launch: only the configurations it is built for
      const int ci = find_cfg(cd_.T, cd_.M);
      if (ci < 0 || !g_pers[ci][src]) continue;
    }
    Plan* P = nullptr;
    if (get_plan(h, &L2, src, s, &P) != CN_OK) continue;
    UserArgs u;
    if (cn_mode) {
      u.psi = (const cd*)d;
      u.V = op->V;
      u.xg = op->xgrid;
      u.dxs = op->dx_per_system;
      u.vscale = op->v_scale;
      u.E_mat = u.E_rhs = E;
      u.dx = op->dx;
      u.dt = op->dt;
    } else {
      u.a = (const cd*)a;
      u.b = (const cd*)b;
      u.c = (const cd*)c;
      u.d = (const cd*)d;
    }
    u.x = (cd*)x;
    // cn_mode 2: a sequence of kSeq steps in place on x from d, as cn_propagate runs it (one
    // fused pass per step over two-pass plans)
    const FusePlan fz = (cn_mode == 2 && fuse_enabled()) ? fuse_plan(P) : FusePlan();
    auto seq = [&]() -> cn_status {
      UserArgs v = u;
      v.psi = (const cd*)x;
      if (fz.ok) return run_chain(h, P, fz, kSeq, [&](int64_t) { return v; }, nullptr, nullptr, s);
      for (int64_t k = 0; k < kSeq; ++k) {
        const cn_status r = run_plan(h, P, v, s);
        if (r != CN_OK) return r;
      }
      return CN_OK;
    };
    std::vector<float> ts;
    bool ok = true;
    for (int r = 0; r < 7 && ok; ++r) {
      if (cn_mode == 2 &&
          hipMemcpyAsync(x, d, (size_t)span * sizeof(cd), hipMemcpyDeviceToDevice, s) != hipSuccess)
        ok = false;
      if (ok && hipEventRecord(e0, s) != hipSuccess) ok = false;
      if (ok && (cn_mode == 2 ? seq() : run_plan(h, P, u, s)) != CN_OK) ok = false;
      if (ok && hipEventRecord(e1, s) != hipSuccess) ok = false;
      if (ok && hipEventSynchronize(e1) != hipSuccess) ok = false;
      float ms = 0.f;
      if (ok && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ok = false;
      if (ok && r >= 2) ts.push_back(ms);
    }
    if (!ok) {
      // a candidate that could not run is left out of the report; its launch error is consumed
      // here so that no later HIP call of the caller reports it
      (void)hipGetLastError();
      continue;
    }
    std::sort(ts.begin(), ts.end());
    const float med = ts[ts.size() / 2];
    char line[160];
    const double per = cn_mode == 2 ? (double)med / kSeq : (double)med;  // per step
    if (cd_.T > 0)
      snprintf(line, sizeof(line), "T=%d M=%d: %.4f ms; ", cd_.T, cd_.M, per);
    else
      snprintf(line, sizeof(line), "automatic: %.4f ms; ", per);
    rep += line;
    if (med < best) {
      best = med;
      best_key = plan_key(&L2, src);
      best_T = cd_.T;
      best_M = cd_.M;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_key.empty()) return CN_ERR_UNSUPPORTED;
  h->tuned[plan_key(L, src)] = best_key;
  rep += "chosen: " + h->plans[best_key]->desc;
  if (!h->cache_path.empty()) {
    char v[32];
    snprintf(v, sizeof(v), "%d,%d", best_T, best_M);
    const std::string cls = cache_class(L, src);
    h->cache[cls] = v;
    std::map<std::string, float> ms;
    ms[cls] = best;
    const cn_status cst = cache_store(h, ms);
    if (cst != CN_OK) return cst;
    rep += " (cached)";
  }
  if (report && report_len > 0) snprintf(report, (size_t)report_len, "%s", rep.c_str());
  return CN_OK;
}

namespace {
// The reverse mode of cn_propagate.  The states of each segment of K steps come either from a
// checkpoint (ckpt: recomputed forward) or, with psi_T instead, from the state at the
// segment's end (rebuilt backwards: psi_k = (1 - i tau H_k)^{-1} (1 + i tau H_k) psi_{k+1}, a
// CN step with dt -> -dt, the inverse of the forward step for a real potential).
cn_status propagate_adjoint_impl(cn_handle_t h, const cn_layout* L, const cn_operator* op,
                                 int64_t nsteps, const double* E, const void* ckpt,
                                 const void* psi_T, int64_t K, void* seg, void* g,
                                 double* dV_accum, double* dE, cn_stream_t stream) {
  if (!h || !L || (!ckpt == !psi_T) || !seg || !g || nsteps < 1 || K < 1)
    return CN_ERR_INVALID_ARG;
  if (L && L->shared_coefficients == 1) return CN_ERR_UNSUPPORTED;
  if (L->offsets) return CN_ERR_UNSUPPORTED;
  cn_status st = check_op(op);
  if (st != CN_OK) return st;
  if (dE && !op->xgrid) return CN_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  Plan* P = nullptr;
  bool fused = true;
  st = cn_plan(h, L, op, s, &P, &fused);
  if (st != CN_OK) return st;
  if (!fused) return CN_ERR_UNSUPPORTED;
  cd* segs = (cd*)seg;
  const int64_t span = P->span;
  // dE: every step of a segment writes its row of per-tile partials; one launch per segment
  // sums the rows (the same fixed order as one sum per step)
  double* part = nullptr;
  if (dE) {
    const size_t need = (size_t)std::min<int64_t>(K, nsteps) * (size_t)P->ntiles1;
    if (h->rows_cap < need) {
      if (capturing(s)) return CN_ERR_NOT_RESERVED;
      size_t bytes = h->rows_cap * sizeof(double);
      void* p = h->rows_buf;
      st = regrow(h, &p, &bytes, need * sizeof(double));
      h->rows_buf = (double*)p;
      h->rows_cap = bytes / sizeof(double);
      if (st != CN_OK) return st;
    }
    part = h->rows_buf;
  }
  auto Ek = [&](int64_t k) { return E ? E[k] : 0.0; };
  const int64_t nseg = (nsteps + K - 1) / K;
  auto k0_of = [&](int64_t sg) { return sg * K; };
  auto k1_of = [&](int64_t sg) { return std::min(nsteps, sg * K + K); };
  // recompute segment sg forward from its checkpoint into buf (its K+1 states): a fused chain
  // on the second workspace when there is one, else step by step
  const FusePlan fzr = fuse_enabled() ? fuse_plan(P) : FusePlan();
  // rebuild segment sg backwards into buf from psi at its end: psi_T for the last segment, else
  // the first state of segment sg+1 (held in src_of(sg), which stays valid until that
  // segment's recursion has finished, after this rebuild)
  std::function<const cd*(int64_t)> src_of;  // set once the segment buffers are known
  auto rebuild = [&](int64_t sg, cd* buf, void* ws, hipStream_t st) -> cn_status {
    const int64_t k0 = k0_of(sg), k1 = k1_of(sg), m = k1 - k0;
    const cd* end = (sg == nseg - 1) ? (const cd*)psi_T : src_of(sg);
    HIP_TRY(hipMemcpyAsync(buf + m * span, end, span * sizeof(cd), hipMemcpyDeviceToDevice, st));
    auto bargs = [&](int64_t i) {
      UserArgs u = cn_args(op, Ek(k1 - 1 - i), buf + (m - i) * span, buf + (m - i - 1) * span);
      u.dt = -op->dt;
      return u;
    };
    if (fzr.ok && ws && m >= 2) return run_chain(h, P, fzr, m, bargs, nullptr, nullptr, st, ws);
    for (int64_t i = 0; i < m; ++i) {
      cn_status r = run_plan(h, P, bargs(i), st, ws);
      if (r != CN_OK) return r;
    }
    return CN_OK;
  };
  auto recompute = [&](int64_t sg, cd* buf, void* ws, hipStream_t st) -> cn_status {
    const int64_t k0 = k0_of(sg), k1 = k1_of(sg);
    if (psi_T) return rebuild(sg, buf, ws, st);
    HIP_TRY(hipMemcpyAsync(buf, (const cd*)ckpt + sg * span, span * sizeof(cd),
                           hipMemcpyDeviceToDevice, st));
    if (fzr.ok && ws && k1 - k0 >= 2) {
      auto rargs = [&](int64_t i) {
        return cn_args(op, Ek(k0 + i), buf + i * span, buf + (i + 1) * span);
      };
      return run_chain(h, P, fzr, k1 - k0, rargs, nullptr, nullptr, st, ws);
    }
    for (int64_t k = k0; k < k1; ++k) {
      const UserArgs u = cn_args(op, Ek(k), buf + (k - k0) * span, buf + (k - k0 + 1) * span);
      cn_status r = run_plan(h, P, u, st, ws);
      if (r != CN_OK) return r;
    }
    return CN_OK;
  };
  // The second workspace keeps the recompute off the recursion's workspace (the fused chain
  // holds its next step's slots and edge rows there across steps); overlapped, the second
  // segment buffer holds the next segment.  Both are allocated outside graph capture only.
  const bool cap = capturing(s);
  const bool overlap = nseg >= 2 && !cap && bwd_overlap_enabled();
  if (!cap) {
    const size_t sb = overlap ? (size_t)(std::min(K, nsteps) + 1) * (size_t)span * sizeof(cd) : 0;
    if (h->ws2_size < P->ws_bytes) {
      st = regrow(h, &h->ws2, &h->ws2_size, P->ws_bytes);
      if (st != CN_OK) return st;
    }
    if (h->seg2_bytes < sb) {
      st = regrow(h, &h->seg2, &h->seg2_bytes, sb);
      if (st != CN_OK) return st;
    }
    if (overlap && !h->aux) {
      HIP_TRY(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
      for (hipEvent_t& e : h->ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
  }
  const FusePlan fz = fuse_enabled() ? fuse_plan(P) : FusePlan();
  const bool chain = fz.ok && h->ws2 && h->ws2_size >= P->ws_bytes;
  cd* bufs[2] = {segs, overlap ? (cd*)h->seg2 : segs};
  auto buf_of = [&](int64_t sg) { return overlap ? bufs[(nseg - 1 - sg) & 1] : segs; };
  src_of = [&](int64_t sg) -> const cd* { return buf_of(sg + 1); };
  hipEvent_t start = h->ev[0], rec_done[2] = {h->ev[1], h->ev[2]},
             adj_done[2] = {h->ev[3], h->ev[4]};
  // The recursion runs on g in place, step k = nsteps-1 .. 0 (chain step i = nsteps-1-k):
  //   g_k = B_k^H lambda_k with lambda_k = T_k^{-H} g_{k+1}, i.e.
  //   g_k = T_k^{-H} B_k^H g_{k+1}  (the two factors commute: B_k = 2 - T_k),
  // a CN step with dt -> -dt (and W -> -W: T_k^H = 1 + tau W - i tau (...), B_k^H = 1 - tau W +
  // i tau (...)) and E_k on both sides; for a real potential T_k^H = B_k, B_k^H = T_k, and
  //   lambda_k = (g_k + g_{k+1}) / 2   (T_k^H + B_k^H = 2),
  // which the store of step k forms for the accumulation.  g_N is the gradient at the final
  // state; g_0, the result, is the gradient at the initial one.
  auto args = [&](int64_t i) {
    const int64_t k = nsteps - 1 - i, sg = k / K, k0 = k0_of(sg);
    const cd* buf = buf_of(sg);
    UserArgs u = cn_args(op, Ek(k), (const cd*)g, (cd*)g);
    u.dt = -op->dt;
    u.wscale = -1.0;
    u.acc_pa = buf + (k - k0) * span;
    u.acc_pb = buf + (k - k0 + 1) * span;
    u.acc_dV = dV_accum;
    u.acc_part = dE ? part + (k - k0) * P->ntiles1 : nullptr;
    u.acc_tau = 0.5 * op->dt;
    u.acc_half = 1;
    return u;
  };
  // entering segment sg (at its last step): its states must be there.  Overlapped, the
  // recompute of segment sg-1 starts on the second stream once segment sg+1 has released the
  // buffer it will use; serially the segment is recomputed here.
  auto before = [&](int64_t i) -> cn_status {
    const int64_t k = nsteps - 1 - i, sg = k / K;
    if (k != k1_of(sg) - 1) return CN_OK;
    if (overlap) {
      const int b = (int)((nseg - 1 - sg) & 1);
      if (sg >= 1) {
        if (sg + 1 <= nseg - 1) HIP_TRY(hipStreamWaitEvent(h->aux, adj_done[1 - b], 0));
        cn_status r = recompute(sg - 1, bufs[1 - b], h->ws2, h->aux);
        if (r != CN_OK) return r;
        HIP_TRY(hipEventRecord(rec_done[1 - b], h->aux));
      }
      HIP_TRY(hipStreamWaitEvent(s, rec_done[b], 0));
      return CN_OK;
    }
    return recompute(sg, segs, chain ? h->ws2 : nullptr, s);
  };
  // leaving segment sg (after its first step): its dE rows are summed (one launch, the fixed
  // order of one sum per step) and its buffer is released
  auto after = [&](int64_t i) -> cn_status {
    const int64_t k = nsteps - 1 - i, sg = k / K, k0 = k0_of(sg);
    if (k != k0) return CN_OK;
    if (dE) {
      const cn_status r = launch_sum_partials(part, P->ntiles1, dE + k0, k1_of(sg) - k0, s);
      if (r != CN_OK) return r;
    }
    if (overlap) HIP_TRY(hipEventRecord(adj_done[(nseg - 1 - sg) & 1], s));
    return CN_OK;
  };
  if (overlap) {
    HIP_TRY(hipEventRecord(start, s));
    HIP_TRY(hipStreamWaitEvent(h->aux, start, 0));
    st = recompute(nseg - 1, bufs[0], h->ws2, h->aux);
    if (st != CN_OK) return st;
    HIP_TRY(hipEventRecord(rec_done[0], h->aux));
  }
  if (chain) return run_chain(h, P, fz, nsteps, args, before, after, s);
  for (int64_t i = 0; i < nsteps; ++i) {
    if ((st = before(i)) != CN_OK) return st;
    if ((st = run_plan(h, P, args(i), s)) != CN_OK) return st;
    if ((st = after(i)) != CN_OK) return st;
  }
  return CN_OK;
}
}  // namespace

cn_status cn_propagate_adjoint(cn_handle_t h, const cn_layout* L, const cn_operator* op,
                               int64_t nsteps, const double* E, const void* ckpt, int64_t K,
                               void* seg, void* g, double* dV_accum, double* dE,
                               cn_stream_t stream) {
  if (!ckpt) return CN_ERR_INVALID_ARG;
  return propagate_adjoint_impl(h, L, op, nsteps, E, ckpt, nullptr, K, seg, g, dV_accum, dE,
                                stream);
}

cn_status cn_propagate_adjoint_reconstruct(cn_handle_t h, const cn_layout* L,
                                           const cn_operator* op, int64_t nsteps,
                                           const double* E, const void* psi_T, int64_t K,
                                           void* seg, void* g, double* dV_accum, double* dE,
                                           cn_stream_t stream) {
  if (!psi_T || !op) return CN_ERR_INVALID_ARG;
  if (op->absorb) return CN_ERR_UNSUPPORTED;  // the backward step would amplify
  return propagate_adjoint_impl(h, L, op, nsteps, E, nullptr, psi_T, K, seg, g, dV_accum, dE,
                                stream);
}

cn_status cn_handle_info(cn_handle_t h, int64_t* device_bytes, int64_t* retired_buffers,
                         int32_t* captured) {
  if (!h) return CN_ERR_INVALID_ARG;
  if (device_bytes) {
    size_t b = h->ws_size + h->ws2_size + h->seg2_bytes + h->mat_size + h->rad_size +
               h->rows_cap * sizeof(double);
    for (const auto& kv : h->plans) b += kv.second->tables_bytes;
    *device_bytes = (int64_t)b;
  }
  if (retired_buffers) *retired_buffers = (int64_t)h->retired.size();
  if (captured) *captured = h->captured ? 1 : 0;
  return CN_OK;
}

cn_status cn_radial_step(cn_handle_t h, const cn_radial* op, double E, const void* psi_in,
                         void* psi_out, cn_stream_t stream) {
  if (!h || !op || !op->V || !psi_in || !psi_out) return CN_ERR_INVALID_ARG;
  if (op->nr < 1 || op->nl < 1 || op->l0 < 0 || !(op->dr > 0.0) || !(op->dt == op->dt) ||
      !(E == E))
    return CN_ERR_INVALID_ARG;
  if (op->nr > ((int64_t)1 << 40) / op->nl) return CN_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  const int64_t nr = op->nr, nl = op->nl, tot = nr * nl;
  // the field part: at every r_j the CN step in l; its systems (one per r_j) are interleaved
  cn_layout Ll{};
  Ll.n = nl;
  Ll.batch = nr;
  Ll.elem_stride = nr;
  Ll.batch_stride = 1;
  // fused when the column kernels take the layout (at least 64 radial points): the rows are
  // built from psi in-kernel; otherwise materialised into the handle buffer
  Plan* Pc = nullptr;
  bool fused = false;
  if (E != 0.0) {
    const cn_status sp = get_plan(h, &Ll, nsd::SRC_LCOUP, s, &Pc);
    if (sp == CN_OK)
      fused = true;
    else if (sp != CN_ERR_UNSUPPORTED)
      return sp;
  }
  const size_t vbytes = ((size_t)tot * sizeof(double) + 255) & ~size_t(255);
  const size_t need = vbytes + (fused || E == 0.0 ? 0 : 4 * (size_t)tot * sizeof(cd));
  if (h->rad_size < need) {
    if (capturing(s)) return CN_ERR_NOT_RESERVED;
    const cn_status st = regrow(h, &h->rad, &h->rad_size, need);
    if (st != CN_OK) return st;
  }
  double* veff = (double*)h->rad;
  cd* m = (cd*)((char*)h->rad + vbytes);
  // radial part: V(r) + l(l+1)/(2 r^2) per wave, then the CN step of every wave in r
  nsd::AuxArgs X{};
  X.n = nr;
  X.batch = nl;
  X.total = tot;
  X.V = op->V;
  X.dx = op->dr;
  X.dt = op->dt;
  X.l0 = op->l0;
  X.vscale = 1.0;
  X.wscale = 1.0;
  X.dV = veff;
  cn_status st = launch_aux(aux_fn(nsk::AUX_RADIAL_VEFF), tot, X, s);
  if (st != CN_OK) return st;
  cn_layout Lr{};
  Lr.n = nr;
  Lr.batch = nl;
  Lr.elem_stride = 1;
  Lr.batch_stride = nr;
  cn_operator o{};
  o.V = veff;
  o.v_scale = 1.0;
  o.dx = op->dr;
  o.dt = op->dt;
  st = cn_step(h, &Lr, &o, 0.0, psi_in, psi_out, stream);
  if (st != CN_OK || E == 0.0) return st;
  if (fused) {
    UserArgs u;
    u.psi = (const cd*)psi_out;
    u.x = (cd*)psi_out;
    u.dx = op->dr;
    u.dt = op->dt;
    u.E_mat = E;
    u.l0 = op->l0;
    return run_plan(h, Pc, u, s);
  }
  X.E = E;
  X.psi = (const cd*)psi_out;
  X.a = m;
  X.b = m + tot;
  X.c = m + 2 * tot;
  X.d = m + 3 * tot;
  st = launch_aux(aux_fn(nsk::AUX_RADIAL_COUPLING), tot, X, s);
  if (st != CN_OK) return st;
  return cn_tridiag_solve(h, &Ll, m, m + tot, m + 2 * tot, m + 3 * tot, psi_out, stream);
}

cn_status cn_tune_cache(cn_handle_t h, const char* path) {
  if (!h) return CN_ERR_INVALID_ARG;
  h->cache_path = path ? path : "";
  if (h->cache_path.empty()) {
    h->cache.clear();
    return CN_OK;
  }
  return cache_load(h);
}

cn_status cn_profile(cn_handle_t h, int enable) {
  if (!h) return CN_ERR_INVALID_ARG;
  h->profiling = enable != 0;
  return CN_OK;
}

cn_status cn_profile_report(cn_handle_t h, char* buf, int64_t buflen) {
  if (!h || !buf || buflen < 1) return CN_ERR_INVALID_ARG;
  std::string out;
  cn_status st = CN_OK;
  for (auto& r : h->recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess)
      st = CN_ERR_HIP;
    char line[224];
    snprintf(line, sizeof(line), "%s ms=%.6f\n", r.label.c_str(), (double)ms);
    out += line;
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  h->recs.clear();
  snprintf(buf, (size_t)buflen, "%s", out.c_str());
  return st;
}

cn_status cn_get_status(cn_handle_t h, cn_stream_t stream) {
  if (!h) return CN_ERR_INVALID_ARG;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  int v = 0;
  HIP_TRY(hipMemcpy(&v, h->status, sizeof(int), hipMemcpyDeviceToHost));
  if (v) {
    HIP_TRY(hipMemset(h->status, 0, sizeof(int)));
    return (v & 4) ? CN_ERR_WAIT_TIMEOUT : CN_NUMERICAL_BREAKDOWN;
  }
  return CN_OK;
}

}  // extern "C"
