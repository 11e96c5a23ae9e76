// Host side of the C ABI declared in include/opf.h: validation, the
// CSR-by-node structure, workspace layout, launch sequencing of one
// message-passing iteration (Section 3.2 of arXiv 2410.17203) for one
// instance or a batch of instances, HIP-graph blocks of iterations, the
// solve loop with FP64 polishing, per-kernel event timing and the launch
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/opf.h"
#include "opf_internal.h"

using namespace opf;

namespace {

constexpr size_t kAlign = 256;
// Upper bound of the sweep grid (partials are sized for it); the grid used is
// the number of blocks resident at once on the device times a tuning factor.
constexpr int kMaxSweepBlocks = 8192;

thread_local std::string g_create_error;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int round8(int64_t x) { return int((x + 7) / 8 * 8); }

struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    size_t off = total;
    total += align_up(bytes);
    return off;
  }
};

struct BufOffsets {
  size_t P, Tm, V1, V2, Td, Hd, Tz, U, W, TB;
};
struct StateOffsets {
  BufOffsets buf[2];
  size_t avgW, avgTB, pnc, thnc, vbar, ramp, bat;
  size_t begin, end;
};

struct Timed {
  int kind;
  hipEvent_t a, b;
};

// One loaded instance.
struct Inst {
  int N = 0, T = 0, K = 0, Kp = 0, Kpp = 0, L = 0, G = 0, D = 0, B = 0, Jnc = 0, nR = 0;
  int Ldc = 0;  // DC links
  int n_chg = 0, Zc = 0;  // per-contingency changes; those that take a line out
  uint64_t topo_hash = 0;  // fingerprint of the network's structure
  double eps_eff = 0.0, rms_norm = 1.0;
  Topo topo{};
  Geom geom64{}, geom32{};
  State<double, double> st64{};
  State<float, float> st32{};
  State<float, bf16_t> st32b{};
  Ctl* ctl = nullptr;
  Rec* ring = nullptr;
  size_t state_begin = 0, state_end = 0;  // workspace range of the iterate
};

// Offsets of everything one instance holds in the workspace.
// Snapshot of the iterate of one precision: 17 arrays (line P, Tm, V1, V2,
// outaged half difference, node U, W, thetabar, the two node means, device
// power/phase/phase dual, ramp and battery inner states, DC link half
// differences, half differences of lines taken out by changes), packed.
constexpr int kSnapArrays = 17;
static_assert(kSnapArrays <= kMaxCopy, "snapshot copy list");
struct SnapLayout {
  size_t off[kSnapArrays];
  size_t bytes[kSnapArrays];
  size_t total;
};

// Tape of a forward run: penalty-schedule history, checkpoints every C
// iterations, the final iterate, C per-iteration snapshots of the segment
// being reversed, and the adjoint arrays.
struct TapePlan {
  bool ready = false;
  int n_iters = 0, every = 0, precision = 0;
  char* base = nullptr;
  size_t bytes = 0;
  SnapLayout snap{};
  size_t hist = 0, ckpt = 0, n_ckpt = 0, final_snap = 0, seg = 0;
  size_t masks = 0, mask_words = 0;  // clip masks of every iteration [M][mask_words] (uint32)
  size_t adj_line[2][4] = {}, adj_td[2] = {}, adj_hd[2] = {}, adj_tz[2] = {}, adj_node[2][3] = {};
  size_t gsp = 0, gsb = 0;
  size_t dev[5] = {};
  size_t ramp_adj = 0, bat_adj = 0, gcap = 0, gload = 0, gpmax = 0;
  size_t adj_begin = 0, adj_end = 0;
  size_t total = 0;
};

struct InstPlan {
  size_t ctl, ring;
  size_t line_from, line_to, sus, cap, outage_k, node_lptr, node_lterm, node_nptr, node_nterm, deg,
      inv_deg, hinv_sus,
      nc_node, ramp_idx, gen_c2, gen_c1, gen_pmin, gen_pmax, gen_ramp, load_d, bat_P, bat_dur,
      bat_eta, bat_alpha;
  size_t part_sweep, part_nc;
  size_t clus_n0, tl_ptr, tl, tcsr, line_dc, chg_ptr, chg;
  StateOffsets o64{}, o32{};
};

}  // namespace

struct opf_ctx {
  opf_options opt{};
  std::string err;
  hipStream_t stream = nullptr;
  bool loaded = false;
  bool batch = false;
  std::vector<Inst> inst;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool has64 = false, has32 = false;
  int precision = 0;  // 0 = FP64 iterate active, 1 = FP32
  bool bf16_duals = false;
  int64_t host_iter = 0;
  int max_T = 1;
  // the fixed per-device workspace (opf_load_network_static): the device
  // whose array holds this context's instance, or -1; taken_over is set when
  // another context's static load replaced it
  int static_dev = -1;
  bool taken_over = false;
  // batch work lists (device) and their descriptors per precision
  BatchTab tab64{}, tab32{};
  void* d_descs64 = nullptr;
  void* d_descs32 = nullptr;
  int64_t* d_dev_prefix = nullptr;
  int64_t* d_grp64 = nullptr;
  int64_t* d_grp32 = nullptr;
  int64_t* d_tiles64 = nullptr;
  int64_t* d_tiles32 = nullptr;
  int32_t* d_queue = nullptr;  // work counters of the batched tiled sweep (zero at load)
  // launch tuning
  int lanes_shift = 0;       // lanes per row = natural value << shift (or >>)
  double grid_factor = 1.0;  // sweep grid = resident blocks * factor
  int tile_mode = -1;        // tiled FP32 sweep: -1 by size, 0 off, 1 on
  int tile_groups = 1;       // period groups per work item of the tiled sweep
  // pinned readback buffers
  Ctl* h_ctl = nullptr;
  int h_ctl_count = 0;
  Rec* h_rec = nullptr;
  int32_t* h_int = nullptr;
  // timing
  bool timing = false;
  std::vector<Timed> pending;
  std::vector<hipEvent_t> pool;
  double t_ms[OPF_KERNEL_COUNT] = {0, 0, 0, 0};
  int64_t t_n[OPF_KERNEL_COUNT] = {0, 0, 0, 0};
  // graphs keyed by (precision, length)
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  // record of a forward run for the adjoint
  TapePlan tape{};
  std::vector<Ctl> tape_hist;
  // batch instances left out of the work lists (stopped ones, while opf_solve runs)
  std::vector<char> retired;
};

namespace {

opf_status fail(opf_ctx* c, opf_status s, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_create_error = msg;
  return s;
}

#define HIP_TRY(c, expr)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((c), OPF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

bool finite(double x) { return std::isfinite(x); }

std::string not_loaded_msg(const opf_ctx* c) {
  return c->taken_over ? "no network loaded: another context's opf_load_network_static took over "
                         "this device's fixed workspace"
                       : "no network loaded";
}

// Validates one network against the context's options.
opf_status validate(opf_ctx* c, const opf_network* n) {
  if (!n) return fail(c, OPF_E_INVALID, "network is NULL");
  if (n->N < 1) return fail(c, OPF_E_INVALID, "N must be >= 1");
  if (n->T < 1 || n->T > 256) return fail(c, OPF_E_INVALID, "T must be in [1, 256]");
  if (n->K < 0) return fail(c, OPF_E_INVALID, "K must be >= 0");
  if (n->L < 0 || n->G < 0 || n->D < 0 || n->B < 0)
    return fail(c, OPF_E_INVALID, "device counts must be >= 0");
  const int Kpp = (n->K + 1 + 3) / 4 * 4;
  const bool need64 = c->opt.state_dtype == OPF_F64 || c->opt.polish_fp64;
  if (need64 && Kpp / 2 > kBlock)
    return fail(c, OPF_E_INVALID, "K too large for an FP64 iterate (K+1 <= 512)");
  if (Kpp / 4 > kBlock) return fail(c, OPF_E_INVALID, "K too large (K+1 <= 1024)");
  const int N = n->N, T = n->T;
  auto bad_ptr = [](int count, const void* p) { return count > 0 && p == nullptr; };
  if (bad_ptr(n->L, n->line_from) || bad_ptr(n->L, n->line_to) || bad_ptr(n->L, n->line_sus) ||
      bad_ptr(n->L, n->line_cap) || bad_ptr(n->K, n->outage) || bad_ptr(n->G, n->gen_node) ||
      bad_ptr(n->G, n->gen_c2) || bad_ptr(n->G, n->gen_c1) || bad_ptr(n->G, n->gen_pmin) ||
      bad_ptr(n->G, n->gen_pmax) || bad_ptr(n->G, n->gen_ramp) || bad_ptr(n->D, n->load_node) ||
      bad_ptr(n->D, n->load_d) || bad_ptr(n->B, n->bat_node) || bad_ptr(n->B, n->bat_P) ||
      bad_ptr(n->B, n->bat_dur) || bad_ptr(n->B, n->bat_eta) || bad_ptr(n->B, n->bat_alpha))
    return fail(c, OPF_E_INVALID, "NULL array for a non-empty device class");
  std::vector<int> deg(N, 0);
  auto node_ok = [&](int v) { return v >= 0 && v < N; };
  for (int l = 0; l < n->L; ++l) {
    if (!node_ok(n->line_from[l]) || !node_ok(n->line_to[l]))
      return fail(c, OPF_E_INVALID, "line node index out of range at line " + std::to_string(l));
    const int kind = n->line_kind ? n->line_kind[l] : 0;
    if (kind != 0 && kind != 1)
      return fail(c, OPF_E_INVALID, "line kind must be 0 (AC) or 1 (DC) at line " + std::to_string(l));
    if (kind == 0 && (!(n->line_sus[l] > 0.0) || !finite(n->line_sus[l])))
      return fail(c, OPF_E_INVALID, "line susceptance must be finite and > 0 at line " + std::to_string(l));
    if (!(n->line_cap[l] >= 0.0) || !finite(n->line_cap[l]))
      return fail(c, OPF_E_INVALID, "line capacity must be finite and >= 0 at line " + std::to_string(l));
    deg[n->line_from[l]]++;
    deg[n->line_to[l]]++;
  }
  std::vector<char> seen(std::max(n->L, 1), 0);
  for (int k = 0; k < n->K; ++k) {
    const int o = n->outage[k];
    if (o < -1 || o >= n->L) return fail(c, OPF_E_INVALID, "outage line index out of range");
    if (o >= 0) {
      if (seen[o]) return fail(c, OPF_E_INVALID, "outage lines must be distinct");
      seen[o] = 1;
    }
  }
  if (n->n_chg < 0) return fail(c, OPF_E_INVALID, "n_chg must be >= 0");
  if (n->n_chg > 0 && (!n->chg_k || !n->chg_line || !n->chg_sus || !n->chg_cap))
    return fail(c, OPF_E_INVALID, "NULL array for a non-empty change list");
  {
    std::vector<std::pair<int, int>> pairs;
    pairs.reserve(size_t(n->n_chg));
    for (int i = 0; i < n->n_chg; ++i) {
      const int k = n->chg_k[i], l = n->chg_line[i];
      if (k < 1 || k > n->K) return fail(c, OPF_E_INVALID, "change contingency out of range (1..K)");
      if (l < 0 || l >= n->L) return fail(c, OPF_E_INVALID, "change line index out of range");
      if (n->outage[k - 1] == l)
        return fail(c, OPF_E_INVALID, "a change repeats its contingency's outage line");
      const bool dc = n->line_kind && n->line_kind[l] == 1;
      if (!(n->chg_cap[i] >= 0.0) || !finite(n->chg_cap[i]) ||
          (!dc && (!(n->chg_sus[i] >= 0.0) || !finite(n->chg_sus[i]))))
        return fail(c, OPF_E_INVALID, "a change needs finite sus >= 0 and cap >= 0");
      pairs.emplace_back(k, l);
    }
    std::sort(pairs.begin(), pairs.end());
    if (std::adjacent_find(pairs.begin(), pairs.end()) != pairs.end())
      return fail(c, OPF_E_INVALID, "a (contingency, line) pair is changed twice");
  }
  for (int g = 0; g < n->G; ++g) {
    if (!node_ok(n->gen_node[g])) return fail(c, OPF_E_INVALID, "generator node out of range");
    deg[n->gen_node[g]]++;
    if (!(n->gen_c2[g] >= 0.0) || !finite(n->gen_c2[g]) || !finite(n->gen_c1[g]))
      return fail(c, OPF_E_INVALID, "generator costs must be finite with c2 >= 0");
    if (std::isnan(n->gen_ramp[g])) return fail(c, OPF_E_INVALID, "generator ramp is NaN");
    for (int t = 0; t < T; ++t) {
      const double lo = n->gen_pmin[size_t(g) * T + t], hi = n->gen_pmax[size_t(g) * T + t];
      if (!finite(lo) || !finite(hi) || lo > hi)
        return fail(c, OPF_E_INVALID, "generator limits must be finite with pmin <= pmax");
    }
  }
  for (int d = 0; d < n->D; ++d) {
    if (!node_ok(n->load_node[d])) return fail(c, OPF_E_INVALID, "load node out of range");
    deg[n->load_node[d]]++;
    for (int t = 0; t < T; ++t) {
      const double v = n->load_d[size_t(d) * T + t];
      if (!finite(v) || v < 0.0) return fail(c, OPF_E_INVALID, "load demand must be finite and >= 0");
    }
  }
  for (int b = 0; b < n->B; ++b) {
    if (!node_ok(n->bat_node[b])) return fail(c, OPF_E_INVALID, "battery node out of range");
    deg[n->bat_node[b]]++;
    if (!(n->bat_P[b] >= 0.0) || !finite(n->bat_P[b]) || !(n->bat_dur[b] >= 0.0) ||
        !finite(n->bat_dur[b]) || !(n->bat_eta[b] > 0.0) || !(n->bat_eta[b] <= 1.0) ||
        !(n->bat_alpha[b] >= 0.0) || !finite(n->bat_alpha[b]))
      return fail(c, OPF_E_INVALID, "battery needs P >= 0, dur >= 0, 0 < eta <= 1, alpha >= 0");
  }
  for (int v = 0; v < N; ++v)
    if (deg[v] < 1) return fail(c, OPF_E_INVALID, "node " + std::to_string(v) + " has no terminal");
  return OPF_OK;
}

// FNV-1a over the structure of a network (line ends and kinds, outages,
// changed (contingency, line) pairs, device nodes): an exported iterate can
// only be imported into a network with the same structure, whose scaled
// prices then keep their invariants (one price per node, phase duals summing
// to zero at every node).
uint64_t topology_hash(const opf_network* n) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t bytes) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < bytes; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  };
  const int32_t sizes[7] = {n->N, n->T, n->K, n->L, n->G, n->D, n->B};
  mix(sizes, sizeof(sizes));
  if (n->L > 0) {
    mix(n->line_from, size_t(n->L) * 4);
    mix(n->line_to, size_t(n->L) * 4);
    if (n->line_kind) mix(n->line_kind, size_t(n->L) * 4);
  }
  if (n->K > 0) mix(n->outage, size_t(n->K) * 4);
  if (n->n_chg > 0) {
    mix(n->chg_k, size_t(n->n_chg) * 4);
    mix(n->chg_line, size_t(n->n_chg) * 4);
  }
  if (n->G > 0) mix(n->gen_node, size_t(n->G) * 4);
  if (n->D > 0) mix(n->load_node, size_t(n->D) * 4);
  if (n->B > 0) mix(n->bat_node, size_t(n->B) * 4);
  return h;
}

void set_sizes(Inst& s, const opf_network* n) {
  s.N = n->N;
  s.T = n->T;
  s.K = n->K;
  s.Kp = n->K + 1;
  s.Kpp = (s.Kp + 3) / 4 * 4;
  s.L = n->L;
  s.G = n->G;
  s.D = n->D;
  s.B = n->B;
  s.Jnc = n->G + n->D + n->B;
  s.Ldc = 0;
  if (n->line_kind)
    for (int l = 0; l < n->L; ++l) s.Ldc += n->line_kind[l] == 1;
  s.n_chg = n->n_chg;
  s.topo_hash = topology_hash(n);
  s.Zc = 0;
  for (int i = 0; i < n->n_chg; ++i) {
    const int l = n->chg_line[i];
    const bool dc = n->line_kind && n->line_kind[l] == 1;
    if (!dc && n->chg_sus[i] == 0.0) s.Zc++;
  }
  s.nR = 0;
  if (n->T > 1)
    for (int g = 0; g < n->G; ++g)
      if (n->gen_ramp[g] > 0.0 && std::isfinite(n->gen_ramp[g])) s.nR++;
}

// Launch geometry of one instance for 16-byte vectors of `vec` elements;
// lanes_shift scales the lanes per row (tuning), resident caps the grid.
void make_geom(const opf_ctx* c, const Inst& s, int vec, int resident, int resident_tile,
               Geom& g) {
  g.nv = s.Kpp / vec;
  g.n_nc_blocks = (s.Jnc + 3) / 4;
  int lpr = 1;
  while (lpr < g.nv && lpr < kWave) lpr *= 2;
  if (c->lanes_shift > 0)
    lpr = std::min(kWave, lpr << c->lanes_shift);
  else if (c->lanes_shift < 0)
    lpr = std::max(1, lpr >> (-c->lanes_shift));
  g.lanes_per_row = lpr;
  g.rows_per_grp = (kBlock / kWave) * (kWave / lpr);
  const int64_t NT = int64_t(s.N) * s.T;
  g.n_grps = (NT + g.rows_per_grp - 1) / g.rows_per_grp;
  g.n_sweep_blocks = std::max(8, round8(std::min<int64_t>(g.n_grps, kMaxSweepBlocks)));
  if (resident >= 8) {
    const int cap = std::min(kMaxSweepBlocks, std::max(8, int(resident * c->grid_factor) / 8 * 8));
    g.n_sweep_blocks = std::max(8, std::min(g.n_sweep_blocks, cap));
  }
  g.tile_blocks = 0;
  g.tile_run = (vec == 2 ? tile_group_periods<double>(s.Kpp) : tile_group_periods<float>(s.Kpp)) *
               std::max(1, c->tile_groups);
  // the tiled sweep whenever the clusters exist (measured faster than the
  // node rows at every size from 30 nodes up); tile_mode 0 forces node rows
  const bool want_tiles = c->tile_mode != 0;
  if (!c->batch && want_tiles && s.topo.Q > 0 && resident_tile >= 8) {
    const int64_t items = int64_t((s.T + g.tile_run - 1) / g.tile_run) * s.topo.Q;
    const int cap = std::min(kMaxSweepBlocks,
                             std::max(8, int(resident_tile * c->grid_factor) / 8 * 8));
    g.tile_blocks = std::max(8, std::min(cap, round8(items)));
  }
  g.n_part = g.tile_blocks > 0 ? g.tile_blocks : g.n_sweep_blocks;
  g.inner_iters = c->opt.inner_iters;
  g.omega_scale = c->opt.inner_omega_scale;
}

template <typename R, typename VT>
void state_offsets(const Inst& s, Layout& lay, StateOffsets& o) {
  const size_t line = size_t(s.L) * s.T * s.Kpp;
  const size_t node = size_t(s.N) * s.T * s.Kpp;
  o.begin = lay.total;
  for (int i = 0; i < 2; ++i) {
    BufOffsets& b = o.buf[i];
    b.P = lay.take(line * sizeof(R));
    b.Tm = lay.take(line * sizeof(R));
    b.V1 = lay.take(line * sizeof(VT));
    b.V2 = lay.take(line * sizeof(VT));
    b.Td = lay.take(size_t(s.T) * s.Kpp * sizeof(R));
    b.Hd = lay.take(size_t(s.Ldc) * s.T * s.Kpp * sizeof(R));
    b.Tz = lay.take(size_t(s.Zc) * s.T * sizeof(R));
    b.U = lay.take(node * sizeof(R));
    b.W = lay.take(node * sizeof(R));
    b.TB = lay.take(node * sizeof(R));
  }
  o.avgW = lay.take(size_t(s.N) * s.T * sizeof(R));
  o.avgTB = lay.take(size_t(s.N) * s.T * sizeof(R));
  const size_t nc = size_t(s.Jnc) * s.T;
  o.pnc = lay.take(nc * sizeof(R));
  o.thnc = lay.take(nc * sizeof(R));
  o.vbar = lay.take(nc * sizeof(R));
  o.ramp = lay.take(4 * size_t(s.nR) * s.T * sizeof(R));
  o.bat = lay.take(6 * size_t(s.B) * s.T * sizeof(R));
  o.end = lay.total;
}

template <typename R, typename VT>
State<R, VT> state_ptrs(char* ws, const StateOffsets& o) {
  State<R, VT> st;
  for (int i = 0; i < 2; ++i) {
    const BufOffsets& b = o.buf[i];
    Buf<R, VT>& d = st.buf[i];
    d.P = reinterpret_cast<R*>(ws + b.P);
    d.Tm = reinterpret_cast<R*>(ws + b.Tm);
    d.V1 = reinterpret_cast<VT*>(ws + b.V1);
    d.V2 = reinterpret_cast<VT*>(ws + b.V2);
    d.Td = reinterpret_cast<R*>(ws + b.Td);
    d.Hd = reinterpret_cast<R*>(ws + b.Hd);
    d.Tz = reinterpret_cast<R*>(ws + b.Tz);
    d.U = reinterpret_cast<R*>(ws + b.U);
    d.W = reinterpret_cast<R*>(ws + b.W);
    d.TB = reinterpret_cast<R*>(ws + b.TB);
  }
  st.avgW = reinterpret_cast<R*>(ws + o.avgW);
  st.avgTB = reinterpret_cast<R*>(ws + o.avgTB);
  st.pnc = reinterpret_cast<R*>(ws + o.pnc);
  st.thnc = reinterpret_cast<R*>(ws + o.thnc);
  st.vbar = reinterpret_cast<R*>(ws + o.vbar);
  st.ramp_st = reinterpret_cast<R*>(ws + o.ramp);
  st.bat_st = reinterpret_cast<R*>(ws + o.bat);
  return st;
}

void plan_instance(const opf_ctx* c, const Inst& s, Layout& L, InstPlan& p) {
  p.ctl = L.take(sizeof(Ctl));
  p.ring = L.take(sizeof(Rec) * kRing);
  const size_t Li = size_t(s.L), Ni = size_t(s.N), Gi = size_t(s.G), T = size_t(s.T);
  p.line_from = L.take(Li * 4);
  p.line_to = L.take(Li * 4);
  p.sus = L.take(Li * 8);
  p.cap = L.take(Li * 8);
  p.outage_k = L.take(size_t(s.Kpp) * 4);
  p.node_lptr = L.take((Ni + 1) * 4);
  p.node_lterm = L.take(4 * Li * 4);
  p.node_nptr = L.take((Ni + 1) * 4);
  p.node_nterm = L.take(size_t(s.Jnc) * 4);
  p.deg = L.take(Ni * 8);
  p.inv_deg = L.take(Ni * 8);
  p.hinv_sus = L.take(Li * 8);
  p.clus_n0 = L.take((Ni + 1) * 4);
  p.tl_ptr = L.take((Ni + 1) * 4);
  p.tl = L.take(2 * Li * 16);
  p.tcsr = L.take(2 * Li * 4);
  p.line_dc = L.take(Li * 4);
  p.chg_ptr = L.take((Li + 1) * 4);
  p.chg = L.take(size_t(s.n_chg) * sizeof(LineChg));
  p.nc_node = L.take(size_t(s.Jnc) * 4);
  p.ramp_idx = L.take(Gi * 4);
  p.gen_c2 = L.take(Gi * 8);
  p.gen_c1 = L.take(Gi * 8);
  p.gen_pmin = L.take(Gi * T * 8);
  p.gen_pmax = L.take(Gi * T * 8);
  p.gen_ramp = L.take(Gi * 8);
  p.load_d = L.take(size_t(s.D) * T * 8);
  p.bat_P = L.take(size_t(s.B) * 8);
  p.bat_dur = L.take(size_t(s.B) * 8);
  p.bat_eta = L.take(size_t(s.B) * 8);
  p.bat_alpha = L.take(size_t(s.B) * 8);
  // residual partials: per sweep block (single instance) or per (row group,
  // wave) (batch, at most one per row plus a block); per device block or per
  // device
  const size_t NT = Ni * T;
  p.part_sweep = L.take(std::max<size_t>(kMaxSweepBlocks, NT + kBlock) * 5 * 8);
  p.part_nc = L.take(std::max<size_t>(s.Jnc, 1) * 2 * 8);
  const bool has32 = c->opt.state_dtype == OPF_F32;
  const bool has64 = !has32 || c->opt.polish_fp64;
  if (has64) state_offsets<double, double>(s, L, p.o64);
  if (has32) {
    if (c->opt.dual_dtype == OPF_BF16)
      state_offsets<float, bf16_t>(s, L, p.o32);
    else
      state_offsets<float, float>(s, L, p.o32);
  }
}

struct BatchPlan {
  size_t descs64, descs32, dev_prefix, grp64, grp32, tiles64, tiles32, queue;
};

void plan_batch(int count, Layout& L, BatchPlan& b) {
  b.descs64 = L.take(sizeof(KArgs<double, double>) * count);
  b.descs32 = L.take(sizeof(KArgs<float, float>) * count);
  b.dev_prefix = L.take(sizeof(int64_t) * (count + 1));
  b.grp64 = L.take(sizeof(int64_t) * (count + 1));
  b.grp32 = L.take(sizeof(int64_t) * (count + 1));
  b.tiles64 = L.take(sizeof(int64_t) * (count + 1));
  b.tiles32 = L.take(sizeof(int64_t) * (count + 1));
  b.queue = L.take(sizeof(int32_t) * 9);  // work counters [8], rescale flag
}

template <typename R, typename VT>
KArgs<R, VT> kargs(const Inst& s, const State<R, VT>& st, const Geom& g) {
  KArgs<R, VT> a;
  a.tp = s.topo;
  a.st = st;
  a.g = g;
  return a;
}

hipEvent_t get_event(opf_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs fn (which enqueues one kernel) bracketed by timing events if enabled.
template <typename Fn>
void timed(opf_ctx* c, int kind, Fn fn, bool capturing) {
  if (!c->timing || capturing) {
    fn();
    return;
  }
  hipEvent_t a = get_event(c), b = get_event(c);
  if (!a || !b) {
    fn();
    return;
  }
  (void)hipEventRecord(a, c->stream);
  fn();
  (void)hipEventRecord(b, c->stream);
  c->pending.push_back({kind, a, b});
}

bool adapt_after(const opf_ctx* c, int64_t iter_index) {
  const int ae = c->opt.adapt_every;
  return ae > 0 && (iter_index + 1) % ae == 0;
}

template <typename R, typename VT>
void enqueue_iter(opf_ctx* c, const KArgs<R, VT>& a, int64_t iter_index, bool capturing) {
  timed(c, OPF_KERNEL_DEVICES, [&] { launch_devices(a, c->stream); }, capturing);
  timed(c, OPF_KERNEL_SWEEP, [&] { launch_sweep(a, c->stream); }, capturing);
  timed(c, OPF_KERNEL_FINALIZE, [&] { launch_finalize(a, c->stream); }, capturing);
  if (adapt_after(c, iter_index))
    timed(c, OPF_KERNEL_RESCALE, [&] { launch_rescale(a, c->stream); }, capturing);
}

template <typename R, typename VT>
void enqueue_batch_iter(opf_ctx* c, const BatchTab& tab, int64_t iter_index, bool capturing) {
  timed(c, OPF_KERNEL_DEVICES,
        [&] { launch_batch_iter_devices<R, VT>(tab, c->max_T, c->stream); }, capturing);
  timed(c, OPF_KERNEL_SWEEP, [&] { launch_batch_iter_sweep<R, VT>(tab, c->stream); }, capturing);
  timed(c, OPF_KERNEL_FINALIZE, [&] { launch_batch_iter_finalize<R, VT>(tab, c->stream); },
        capturing);
  if (adapt_after(c, iter_index))
    timed(c, OPF_KERNEL_RESCALE, [&] { launch_batch_iter_rescale<R, VT>(tab, c->stream); },
          capturing);
}

void enqueue_n(opf_ctx* c, int n, bool capturing, int64_t start) {
  for (int i = 0; i < n; ++i) {
    const int64_t it = start + i;
    if (c->batch) {
      if (c->precision == 0)
        enqueue_batch_iter<double, double>(c, c->tab64, it, capturing);
      else if (c->bf16_duals)
        enqueue_batch_iter<float, bf16_t>(c, c->tab32, it, capturing);
      else
        enqueue_batch_iter<float, float>(c, c->tab32, it, capturing);
      continue;
    }
    const Inst& s = c->inst[0];
    if (c->precision == 0)
      enqueue_iter(c, kargs(s, s.st64, s.geom64), it, capturing);
    else if (c->bf16_duals)
      enqueue_iter(c, kargs(s, s.st32b, s.geom32), it, capturing);
    else
      enqueue_iter(c, kargs(s, s.st32, s.geom32), it, capturing);
  }
}

// Copies every instance's control block to the pinned host array.
opf_status read_ctls(opf_ctx* c) {
  for (size_t i = 0; i < c->inst.size(); ++i)
    HIP_TRY(c, hipMemcpyAsync(c->h_ctl + i, c->inst[i].ctl, sizeof(Ctl), hipMemcpyDeviceToHost,
                              c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return OPF_OK;
}

void fill_resid(const Rec& r, opf_resid* o) {
  o->primal_p = r.primal_p;
  o->primal_theta = r.primal_th;
  o->dual_p = r.dual_p;
  o->dual_theta = r.dual_th;
  o->rms_primal = r.rms_primal;
  o->rms_dual = r.rms_dual;
  o->threshold = r.threshold;
  o->objective = r.objective;
  o->rho_p = r.rho_p;
  o->rho_theta = r.rho_th;
  o->converged = r.converged;
  o->precision = r.precision == 0 ? OPF_F64 : OPF_F32;
}

// Last residual record of instance i (control blocks must be fresh).
opf_status last_record(opf_ctx* c, int i, opf_resid* out) {
  std::memset(out, 0, sizeof(*out));
  const Inst& s = c->inst[i];
  const Ctl& h = c->h_ctl[i];
  const int ce = std::max(1, c->opt.check_every);
  const int last = h.iter - h.iter % ce;
  out->iter = h.iter;
  out->rho_p = h.rho_p;
  out->rho_theta = h.rho_th;
  out->threshold = s.eps_eff;
  out->precision = c->precision == 0 ? OPF_F64 : OPF_F32;
  if (last <= 0) return OPF_OK;
  HIP_TRY(c, hipMemcpyAsync(c->h_rec, s.ring + (last - 1) % kRing, sizeof(Rec),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  fill_resid(*c->h_rec, out);
  out->iter = h.iter;
  return OPF_OK;
}

opf_status widen_to_fp64(opf_ctx* c) {
  for (Inst& s : c->inst) {
    KArgs<double, double> dst = kargs(s, s.st64, s.geom64);
    if (c->bf16_duals)
      launch_widen(kargs(s, s.st32b, s.geom32), dst, c->stream);
    else
      launch_widen(kargs(s, s.st32, s.geom32), dst, c->stream);
    HIP_TRY(c, hipGetLastError());
    *c->h_int = 0;
    HIP_TRY(c, hipMemcpyAsync(&s.ctl->precision, c->h_int, sizeof(int32_t),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  c->precision = 0;
  return OPF_OK;
}

// (Re)computes every instance's launch geometry and the batch work lists.
opf_status refresh_geometry(opf_ctx* c) {
  int res64 = 0, res32 = 0, tile64 = 0, tile32 = 0;
  if (!c->batch) {
    tile64 = tile_resident_blocks<double, double>();
    tile32 = c->bf16_duals ? tile_resident_blocks<float, bf16_t>() : tile_resident_blocks<float, float>();
  }
  if (c->batch) {
    res64 = sweep_batch_resident_blocks<double, double>();
    res32 = c->bf16_duals ? sweep_batch_resident_blocks<float, bf16_t>()
                          : sweep_batch_resident_blocks<float, float>();
    tile64 = tile_batch_resident_blocks<double, double>();
    tile32 = c->bf16_duals ? tile_batch_resident_blocks<float, bf16_t>()
                           : tile_batch_resident_blocks<float, float>();
  } else {
    res64 = sweep_resident_blocks<double, double>();
    res32 = c->bf16_duals ? sweep_resident_blocks<float, bf16_t>()
                          : sweep_resident_blocks<float, float>();
  }
  for (Inst& s : c->inst) {
    for (int p = 0; p < 2; ++p) {
      Geom& g = p == 0 ? s.geom64 : s.geom32;
      const Geom keep = g;  // scratch pointers are fixed at load
      make_geom(c, s, p == 0 ? 2 : 4, p == 0 ? res64 : res32, p == 0 ? tile64 : tile32, g);
      g.part_sweep = keep.part_sweep;
      g.part_nc = keep.part_nc;
      g.ctl = keep.ctl;
      g.ring = keep.ring;
    }
  }
  if (!c->batch) return OPF_OK;
  const int n = int(c->inst.size());
  std::vector<int64_t> dev(n + 1, 0), g64(n + 1, 0), g32(n + 1, 0), tiles64(n + 1, 0),
      tiles32(n + 1, 0);
  // estimated work of one tiled-sweep item of each instance (element
  // updates of a cluster's lines and nodes over the item's periods, plus a
  // fixed cost), for XCD ranges of equal work
  std::vector<double> cost64(n), cost32(n);
  // the batch takes the tiled sweep over all instances' tiles when every
  // instance has clusters (unless tile_mode forces node rows)
  bool all_tiles = true;
  std::vector<KArgs<double, double>> d64(n);
  std::vector<KArgs<float, float>> d32(n);
  std::vector<KArgs<float, bf16_t>> d32b(n);
  for (int i = 0; i < n; ++i) {
    const Inst& s = c->inst[i];
    // a retired instance has no work items, device waves or row groups
    const int64_t on = (size_t(i) < c->retired.size() && c->retired[i]) ? 0 : 1;
    dev[i + 1] = dev[i] + on * s.Jnc;
    g64[i + 1] = g64[i] + on * s.geom64.n_grps;
    g32[i + 1] = g32[i] + on * s.geom32.n_grps;
    const int64_t Q = on * s.topo.Q;
    tiles64[i + 1] = tiles64[i] + int64_t((s.T + s.geom64.tile_run - 1) / s.geom64.tile_run) * Q;
    tiles32[i + 1] = tiles32[i] + int64_t((s.T + s.geom32.tile_run - 1) / s.geom32.tile_run) * Q;
    const double per_period = Q > 0 ? double(2 * s.L + s.N) / double(Q) * s.Kpp : 0.0;
    cost64[i] = per_period * s.geom64.tile_run + 4096.0;
    cost32[i] = per_period * s.geom32.tile_run + 4096.0;
    all_tiles = all_tiles && s.topo.Q > 0;  // (of every instance, retired or not)
    d64[i] = kargs(s, s.st64, s.geom64);
    d32[i] = kargs(s, s.st32, s.geom32);
    d32b[i] = kargs(s, s.st32b, s.geom32);
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_descs64, d64.data(), sizeof(KArgs<double, double>) * n,
                            hipMemcpyHostToDevice, c->stream));
  if (c->bf16_duals)
    HIP_TRY(c, hipMemcpyAsync(c->d_descs32, d32b.data(), sizeof(KArgs<float, bf16_t>) * n,
                              hipMemcpyHostToDevice, c->stream));
  else
    HIP_TRY(c, hipMemcpyAsync(c->d_descs32, d32.data(), sizeof(KArgs<float, float>) * n,
                              hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_dev_prefix, dev.data(), sizeof(int64_t) * (n + 1),
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_grp64, g64.data(), sizeof(int64_t) * (n + 1),
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_grp32, g32.data(), sizeof(int64_t) * (n + 1),
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_tiles64, tiles64.data(), sizeof(int64_t) * (n + 1),
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_tiles32, tiles32.data(), sizeof(int64_t) * (n + 1),
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const bool want_tiles = all_tiles && c->tile_mode != 0;
  auto tab = [&](BatchTab& t, const void* descs, const int64_t* grp, int64_t total_grps, int res,
                 int res_tile, const int64_t* d_tiles, const std::vector<int64_t>& tiles,
                 const std::vector<double>& cost) {
    t.descs = descs;
    t.dev_prefix = c->d_dev_prefix;
    t.grp_prefix = grp;
    t.n_inst = n;
    t.any_gen = 0;
    for (const Inst& x : c->inst) t.any_gen |= (x.Ldc > 0 || x.n_chg > 0) ? 1 : 0;
    t.total_dev = dev[n];
    t.total_grps = total_grps;
    int nb = std::max(8, round8(std::min<int64_t>(total_grps, kMaxSweepBlocks)));
    if (res >= 8)
      nb = std::max(8, std::min(nb, std::min(kMaxSweepBlocks,
                                             std::max(8, int(res * c->grid_factor) / 8 * 8))));
    t.n_sweep_blocks = nb;
    t.tile_prefix = d_tiles;
    t.total_tiles = tiles[n];
    t.tile_queue = c->d_queue;
    t.rescale_flag = c->d_queue + 8;
    {
      double total = 0.0;
      for (int i = 0; i < n; ++i) total += cost[i] * double(tiles[i + 1] - tiles[i]);
      t.xcd_bounds[0] = 0;
      int i = 0;
      double before = 0.0;  // work of the instances before i
      for (int x = 1; x < 8; ++x) {
        const double target = total * x / 8.0;
        while (i < n && before + cost[i] * double(tiles[i + 1] - tiles[i]) < target) {
          before += cost[i] * double(tiles[i + 1] - tiles[i]);
          ++i;
        }
        int64_t b = tiles[n];
        if (i < n) b = tiles[i] + int64_t(std::ceil((target - before) / cost[i]));
        t.xcd_bounds[x] = std::min(tiles[n], std::max(t.xcd_bounds[x - 1], b));
      }
      t.xcd_bounds[8] = tiles[n];
    }
    t.tile_blocks = 0;
    if (want_tiles && res_tile >= 8)
      t.tile_blocks = std::max(8, std::min(std::min(kMaxSweepBlocks,
                                                    std::max(8, int(res_tile * c->grid_factor) / 8 * 8)),
                                           round8(tiles[n])));
  };
  tab(c->tab64, c->d_descs64, c->d_grp64, g64[n], res64, tile64, c->d_tiles64, tiles64, cost64);
  tab(c->tab32, c->d_descs32, c->d_grp32, g32[n], res32, tile32, c->d_tiles32, tiles32, cost32);
  return OPF_OK;
}

// Sets which batch instances are left out of the work lists (r empty: none)
// and rebuilds the lists and graphs if that changes.
opf_status set_retired(opf_ctx* c, const std::vector<char>& r) {
  auto any = [](const std::vector<char>& v) {
    for (char x : v)
      if (x) return true;
    return false;
  };
  if (!c->batch || (!any(r) && !any(c->retired)) || r == c->retired) return OPF_OK;
  c->retired = r;
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  return refresh_geometry(c);
}

// Resets every instance to the all-zero start (Section 3.4).
opf_status reset_state(opf_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  // (every launch of the batched tiled sweep is followed by the finalize
  // that zeroes its work counters; zeroed here too, with the rescale flag,
  // outside any graph)
  if (c->batch && c->d_queue)
    HIP_TRY(c, hipMemsetAsync(c->d_queue, 0, sizeof(int32_t) * 9, c->stream));
  for (size_t i = 0; i < c->inst.size(); ++i) {
    Inst& s = c->inst[i];
    if (s.state_end > s.state_begin)
      HIP_TRY(c, hipMemsetAsync(c->ws + s.state_begin, 0, s.state_end - s.state_begin, c->stream));
    Ctl& h = c->h_ctl[i];
    std::memset(&h, 0, sizeof(Ctl));
    h.rho_p = c->opt.rho_p;
    h.rho_th = c->opt.rho_theta;
    h.su = 1.0;
    h.sv = 1.0;
    h.eps_eff = s.eps_eff;
    h.rms_norm = s.rms_norm;
    h.mu = c->opt.mu;
    h.gamma = c->opt.gamma;
    h.adapt_every = c->opt.adapt_every;
    h.check_every = c->opt.check_every;
    h.max_iter = c->opt.max_iter;
    h.min_iter = c->opt.min_iter;
    h.precision = c->has32 ? 1 : 0;
    HIP_TRY(c, hipMemcpyAsync(s.ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->precision = c->has32 ? 1 : 0;
  c->host_iter = 0;
  return OPF_OK;
}

// Validates all networks and lays out the workspace.
// The derived host tables of one network: node CSR over line terminals and
// devices, the tiled sweep's clusters, DC link and change lists.
struct Tables {
  std::vector<int32_t> outage_k, lptr, nptr, lterm, nterm, nc_node, clus_n0, tl_ptr, tl, tcsr,
      ramp_idx, line_dc, chg_ptr;
  std::vector<double> deg, sus;
  std::vector<LineChg> chg;
  bool tiles_ok = false;
  int Q = 0;  // clusters (0: the tiled sweep is not available)
  double load_rms = 1.0;
};

void build_tables(const opf_network* n, const Inst& s, Tables& t) {
  const int N = s.N, T = s.T, L = s.L, G = s.G, D = s.D, B = s.B, Jnc = s.Jnc, Kpp = s.Kpp;
  std::vector<int32_t> outage_k(Kpp, -1);
  for (int k = 1; k <= s.K; ++k) outage_k[k] = n->outage[k - 1];
  // CSR by node: line terminals ordered (terminal 1 by line, then terminal 2
  // by line), then generators, loads, batteries.
  std::vector<int32_t> lptr(N + 1, 0), nptr(N + 1, 0), lterm(4 * size_t(L)), nterm(Jnc), nc_node(Jnc);
  for (int l = 0; l < L; ++l) {
    lptr[n->line_from[l] + 1]++;
    lptr[n->line_to[l] + 1]++;
  }
  for (int v = 0; v < N; ++v) lptr[v + 1] += lptr[v];
  {
    std::vector<int32_t> fill(lptr.begin(), lptr.end() - 1);
    // entry: (2 l + end, node at the other end of the line)
    for (int l = 0; l < L; ++l) {
      const int q = fill[n->line_from[l]]++;
      lterm[2 * size_t(q)] = 2 * l;
      lterm[2 * size_t(q) + 1] = n->line_to[l];
    }
    for (int l = 0; l < L; ++l) {
      const int q = fill[n->line_to[l]]++;
      lterm[2 * size_t(q)] = 2 * l + 1;
      lterm[2 * size_t(q) + 1] = n->line_from[l];
    }
  }
  for (int g = 0; g < G; ++g) nc_node[g] = n->gen_node[g];
  for (int d = 0; d < D; ++d) nc_node[G + d] = n->load_node[d];
  for (int b = 0; b < B; ++b) nc_node[G + D + b] = n->bat_node[b];
  for (int j = 0; j < Jnc; ++j) nptr[nc_node[j] + 1]++;
  for (int v = 0; v < N; ++v) nptr[v + 1] += nptr[v];
  {
    std::vector<int32_t> fill(nptr.begin(), nptr.end() - 1);
    for (int j = 0; j < Jnc; ++j) nterm[fill[nc_node[j]]++] = j;
  }
  std::vector<double> deg(N);
  for (int v = 0; v < N; ++v) deg[v] = double(lptr[v + 1] - lptr[v] + nptr[v + 1] - nptr[v]);
  // Clusters of consecutive nodes for the tiled sweep: at most kTileNodes
  // nodes, kTileLines distinct incident lines and kTileDev devices each
  // (full-size clusters: smaller ones measured slower at every instance
  // size, their fixed per-tile costs dominating).  Per cluster, the
  // lines touching it (first occurrence in node and CSR order) with the
  // cluster-local index of each end inside it and the far node otherwise;
  // per line terminal, its line's index in that table.
  std::vector<int32_t> clus_n0(1, 0), tl_ptr(1, 0), tl, tcsr(2 * size_t(L), 0);
  bool tiles_ok = N > 0;
  {
    const int cmax = kTileNodes;
    std::vector<int32_t> mark(L, -1), pos(L, 0);
    int n0 = 0;
    while (tiles_ok && n0 < N) {
      const int cid = int(clus_n0.size()) - 1;
      int m = n0, cnt = 0, ndev = 0;
      while (m < N && m - n0 < cmax) {
        int add = 0;
        for (int q = lptr[m]; q < lptr[m + 1]; ++q)
          if (mark[lterm[2 * size_t(q)] >> 1] != cid) ++add;
        if (cnt + add > kTileLines) break;
        if (ndev + (nptr[m + 1] - nptr[m]) > kTileDev) break;
        ndev += nptr[m + 1] - nptr[m];
        for (int q = lptr[m]; q < lptr[m + 1]; ++q) mark[lterm[2 * size_t(q)] >> 1] = cid;
        cnt += add;
        ++m;
      }
      if (m == n0) {  // one node with more lines or devices than a tile holds
        tiles_ok = false;
        break;
      }
      const int n1 = m;
      const int base = int(tl.size() / 4);
      for (int v = n0; v < n1; ++v)
        for (int q = lptr[v]; q < lptr[v + 1]; ++q) {
          const int l = lterm[2 * size_t(q)] >> 1, end = lterm[2 * size_t(q)] & 1;
          if (mark[l] != -2 - cid) {
            mark[l] = -2 - cid;
            pos[l] = int(tl.size() / 4) - base;
            const int f = n->line_from[l], h = n->line_to[l];
            const bool fin = f >= n0 && f < n1, hin = h >= n0 && h < n1;
            tl.push_back(l);
            tl.push_back(fin ? f - n0 : -1);
            tl.push_back(hin ? h - n0 : -1);
            tl.push_back(fin && hin ? -1 : (fin ? h : f));
          }
          tcsr[q] = 2 * pos[l] + end;
        }
      n0 = n1;
      clus_n0.push_back(n0);
      tl_ptr.push_back(int(tl.size() / 4));
    }
  }
  std::vector<int32_t> ramp_idx(G, -1);
  {
    int r = 0;
    if (T > 1)
      for (int g = 0; g < G; ++g)
        if (n->gen_ramp[g] > 0.0 && std::isfinite(n->gen_ramp[g])) ramp_idx[g] = r++;
  }
  // DC links: index among them, and a unit susceptance in place of the
  // ignored one so that the unused AC weights stay finite
  std::vector<int32_t> line_dc(L, -1);
  std::vector<double> sus(n->line_sus, n->line_sus + L);
  {
    int m = 0;
    for (int l = 0; l < L; ++l)
      if (n->line_kind && n->line_kind[l] == 1) {
        line_dc[l] = m++;
        sus[l] = 1.0;
      }
  }
  // per-contingency changes: CSR by line, entries by contingency; changes
  // that take an AC line out are numbered (z) in input order
  std::vector<int32_t> chg_ptr(L + 1, 0);
  std::vector<LineChg> chg(size_t(s.n_chg));
  {
    std::vector<int32_t> zid(size_t(s.n_chg), -1);
    int z = 0;
    for (int i = 0; i < s.n_chg; ++i) {
      const int l = n->chg_line[i];
      chg_ptr[l + 1]++;
      if (line_dc[l] < 0 && n->chg_sus[i] == 0.0) zid[i] = z++;
    }
    for (int l = 0; l < L; ++l) chg_ptr[l + 1] += chg_ptr[l];
    std::vector<int32_t> order(size_t(s.n_chg));
    for (int i = 0; i < s.n_chg; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
      return std::make_pair(n->chg_line[a], n->chg_k[a]) < std::make_pair(n->chg_line[b], n->chg_k[b]);
    });
    for (int q = 0; q < s.n_chg; ++q) {
      const int i = order[q];
      chg[q] = LineChg{n->chg_k[i], zid[i], n->chg_sus[i], n->chg_cap[i]};
    }
  }
  double lsum = 0.0;
  for (size_t i = 0; i < size_t(D) * T; ++i) lsum += n->load_d[i] * n->load_d[i];
  const double load_rms = (size_t(D) * T > 0) ? std::sqrt(lsum / double(size_t(D) * T)) : 1.0;

  t.outage_k = std::move(outage_k);
  t.lptr = std::move(lptr);
  t.nptr = std::move(nptr);
  t.lterm = std::move(lterm);
  t.nterm = std::move(nterm);
  t.nc_node = std::move(nc_node);
  t.deg = std::move(deg);
  t.tiles_ok = tiles_ok;
  t.Q = tiles_ok ? int(clus_n0.size()) - 1 : 0;
  t.clus_n0 = std::move(clus_n0);
  t.tl_ptr = std::move(tl_ptr);
  t.tl = std::move(tl);
  t.tcsr = std::move(tcsr);
  t.ramp_idx = std::move(ramp_idx);
  t.line_dc = std::move(line_dc);
  t.sus = std::move(sus);
  t.chg_ptr = std::move(chg_ptr);
  t.chg = std::move(chg);
  t.load_rms = load_rms;
}

// Checks every index of the derived tables that a kernel reads through
// against the range the kernel assumes (host-side bounds check of the
// device tables: node CSR, clusters and their line tables, device, DC link
// and change indices).  Returns an empty string, or what failed.
std::string check_tables(const opf_network* n, const Inst& s, const Tables& t) {
  const int N = s.N, L = s.L, G = s.G, Jnc = s.Jnc, Kpp = s.Kpp;
  auto in = [](int64_t x, int64_t lo, int64_t hi) { return x >= lo && x < hi; };
  auto at = [](const char* what, int64_t i) { return std::string(what) + " at " + std::to_string(i); };
  if (int(t.outage_k.size()) != Kpp) return "outage table size";
  for (int k = 0; k < Kpp; ++k) {
    const int o = t.outage_k[k];
    // (-1 for the base case, the padding, and a contingency that removes no line)
    if (k >= 1 && k <= s.K ? !in(o, -1, L) : o != -1) return at("outage index", k);
  }
  // node CSR over line terminals: entry 2 l + end at the node of that end,
  // with the node at the line's other end
  auto csr_ok = [&](const std::vector<int32_t>& ptr, int64_t total) {
    if (int(ptr.size()) != N + 1 || ptr[0] != 0 || ptr[N] != total) return false;
    for (int v = 0; v < N; ++v)
      if (ptr[v + 1] < ptr[v]) return false;
    return true;
  };
  if (!csr_ok(t.lptr, 2 * int64_t(L))) return "line terminal CSR pointers";
  for (int v = 0; v < N; ++v)
    for (int q = t.lptr[v]; q < t.lptr[v + 1]; ++q) {
      const int e = t.lterm[2 * size_t(q)], far = t.lterm[2 * size_t(q) + 1];
      if (!in(e, 0, 2 * int64_t(L))) return at("line terminal entry", q);
      const int l = e >> 1;
      const bool to_end = e & 1;
      if ((to_end ? n->line_to[l] : n->line_from[l]) != v ||
          (to_end ? n->line_from[l] : n->line_to[l]) != far)
        return at("line terminal ends", q);
    }
  if (!csr_ok(t.nptr, Jnc)) return "device CSR pointers";
  if (int(t.nc_node.size()) != Jnc) return "device node table size";
  for (int j = 0; j < Jnc; ++j)
    if (!in(t.nc_node[j], 0, N)) return at("device node", j);
  for (int v = 0; v < N; ++v)
    for (int q = t.nptr[v]; q < t.nptr[v + 1]; ++q)
      if (!in(t.nterm[q], 0, Jnc) || t.nc_node[t.nterm[q]] != v) return at("device entry", q);
  for (int v = 0; v < N; ++v)
    if (!(t.deg[v] >= 1.0)) return at("node degree", v);
  // clusters of the tiled sweep: consecutive nodes, their lines, and for
  // every line terminal its line's index in the cluster's table
  if (t.tiles_ok) {
    const int Q = t.Q;
    if (Q < 1 || int(t.clus_n0.size()) != Q + 1 || int(t.tl_ptr.size()) != Q + 1)
      return "cluster table sizes";
    if (t.clus_n0[0] != 0 || t.clus_n0[Q] != N || t.tl_ptr[0] != 0 ||
        size_t(t.tl_ptr[Q]) * 4 != t.tl.size())
      return "cluster table ends";
    for (int cq = 0; cq < Q; ++cq) {
      const int n0 = t.clus_n0[cq], n1 = t.clus_n0[cq + 1];
      const int j0 = t.tl_ptr[cq], j1 = t.tl_ptr[cq + 1];
      if (!(n1 > n0 && n1 - n0 <= kTileNodes)) return at("cluster nodes", cq);
      if (!(j1 >= j0 && j1 - j0 <= kTileLines)) return at("cluster lines", cq);
      if (t.lptr[n1] - t.lptr[n0] > 2 * kTileLines) return at("cluster terminals", cq);
      if (t.nptr[n1] - t.nptr[n0] > kTileDev) return at("cluster devices", cq);
      for (int j = j0; j < j1; ++j) {
        const int32_t* e = &t.tl[4 * size_t(j)];
        if (!in(e[0], 0, L)) return at("cluster line", j);
        const int f = n->line_from[e[0]], h = n->line_to[e[0]];
        const bool fin = f >= n0 && f < n1, hin = h >= n0 && h < n1;
        if (e[1] != (fin ? f - n0 : -1) || e[2] != (hin ? h - n0 : -1)) return at("cluster line ends", j);
        if (e[3] != (fin && hin ? -1 : (fin ? h : f)) || !in(e[3], -1, N) || (!fin && !hin))
          return at("cluster far node", j);
      }
      for (int q = t.lptr[n0]; q < t.lptr[n1]; ++q) {
        const int x = t.tcsr[q];
        if (!in(x >> 1, 0, j1 - j0) || t.tl[4 * size_t(j0 + (x >> 1))] != (t.lterm[2 * size_t(q)] >> 1) ||
            (x & 1) != (t.lterm[2 * size_t(q)] & 1))
          return at("cluster terminal", q);
      }
    }
  }
  int nr = 0;
  for (int g = 0; g < G; ++g) {
    if (t.ramp_idx[g] >= 0 && t.ramp_idx[g] != nr++) return at("ramp index", g);
    if (t.ramp_idx[g] < -1) return at("ramp index", g);
  }
  if (nr != s.nR) return "ramp generator count";
  int nd = 0;
  for (int l = 0; l < L; ++l) {
    if (t.line_dc[l] >= 0 && t.line_dc[l] != nd++) return at("DC link index", l);
    if (t.line_dc[l] < -1) return at("DC link index", l);
  }
  if (nd != s.Ldc) return "DC link count";
  if (int(t.chg_ptr.size()) != L + 1 || t.chg_ptr[0] != 0 || t.chg_ptr[L] != s.n_chg)
    return "change CSR pointers";
  for (int l = 0; l < L; ++l) {
    if (t.chg_ptr[l + 1] < t.chg_ptr[l]) return at("change CSR pointers", l);
    for (int q = t.chg_ptr[l]; q < t.chg_ptr[l + 1]; ++q) {
      const LineChg& ch = t.chg[q];
      if (!in(ch.k, 1, s.K + 1) || !in(ch.z, -1, s.Zc)) return at("change entry", q);
      if (q > t.chg_ptr[l] && !(t.chg[q - 1].k < ch.k)) return at("change order", q);
    }
  }
  return std::string();
}

// Validates the networks and sizes their workspace; with tabs, also builds
// and bounds-checks their derived tables (before anything is changed).
opf_status plan_all(opf_ctx* c, const opf_network* nets, int count, std::vector<Inst>& insts,
                    std::vector<InstPlan>& plans, BatchPlan& bp, Layout& lay,
                    std::vector<Tables>* tabs = nullptr) {
  if (count < 1) return fail(c, OPF_E_INVALID, "need at least one network");
  if (!nets) return fail(c, OPF_E_INVALID, "networks are NULL");
  insts.assign(count, Inst());
  plans.assign(count, InstPlan());
  if (tabs) tabs->assign(count, Tables());
  for (int i = 0; i < count; ++i) {
    opf_status s = validate(c, &nets[i]);
    if (s != OPF_OK) {
      if (count > 1) c->err = "instance " + std::to_string(i) + ": " + c->err;
      return s;
    }
    set_sizes(insts[i], &nets[i]);
    if (tabs) {
      build_tables(&nets[i], insts[i], (*tabs)[i]);
      const std::string why = check_tables(&nets[i], insts[i], (*tabs)[i]);
      if (!why.empty())
        return fail(c, OPF_E_INVALID,
                    (count > 1 ? "instance " + std::to_string(i) + ": " : std::string()) +
                        "derived table check failed: " + why);
    }
  }
  if (count > 1) plan_batch(count, lay, bp);
  for (int i = 0; i < count; ++i) plan_instance(c, insts[i], lay, plans[i]);
  return OPF_OK;
}

opf_status workspace_size(opf_ctx* c, const opf_network* nets, int count, size_t* bytes) {
  if (!c || !bytes) return fail(c, OPF_E_INVALID, "NULL argument");
  std::vector<Inst> insts;
  std::vector<InstPlan> plans;
  BatchPlan bp{};
  Layout lay;
  opf_status s = plan_all(c, nets, count, insts, plans, bp, lay);
  if (s != OPF_OK) return s;
  *bytes = lay.total;
  return OPF_OK;
}

// Copies one network's data and derived tables to the device.
opf_status upload_instance(opf_ctx* c, const opf_network* n, Inst& s, const InstPlan& p,
                           const Tables& t) {
  char* ws = c->ws;
  const int N = s.N, T = s.T, L = s.L, G = s.G, D = s.D, B = s.B, Jnc = s.Jnc, Kpp = s.Kpp;
  const auto& outage_k = t.outage_k;
  const auto& lptr = t.lptr;
  const auto& nptr = t.nptr;
  const auto& lterm = t.lterm;
  const auto& nterm = t.nterm;
  const auto& nc_node = t.nc_node;
  const auto& deg = t.deg;
  const auto& clus_n0 = t.clus_n0;
  const auto& tl_ptr = t.tl_ptr;
  const auto& tl = t.tl;
  const auto& tcsr = t.tcsr;
  const auto& ramp_idx = t.ramp_idx;
  const auto& line_dc = t.line_dc;
  const auto& sus = t.sus;
  const auto& chg_ptr = t.chg_ptr;
  const auto& chg = t.chg;
  const bool tiles_ok = t.tiles_ok;
  const double load_rms = t.load_rms;
  s.topo.Q = t.Q;
  auto up = [&](size_t off, const void* src, size_t nbytes) -> hipError_t {
    if (nbytes == 0) return hipSuccess;
    return hipMemcpyAsync(ws + off, src, nbytes, hipMemcpyHostToDevice, c->stream);
  };
  HIP_TRY(c, up(p.line_from, n->line_from, size_t(L) * 4));
  HIP_TRY(c, up(p.line_to, n->line_to, size_t(L) * 4));
  HIP_TRY(c, up(p.sus, sus.data(), size_t(L) * 8));
  HIP_TRY(c, up(p.line_dc, line_dc.data(), size_t(L) * 4));
  HIP_TRY(c, up(p.chg_ptr, chg_ptr.data(), size_t(L + 1) * 4));
  HIP_TRY(c, up(p.chg, chg.data(), chg.size() * sizeof(LineChg)));
  HIP_TRY(c, up(p.cap, n->line_cap, size_t(L) * 8));
  HIP_TRY(c, up(p.outage_k, outage_k.data(), size_t(Kpp) * 4));
  HIP_TRY(c, up(p.node_lptr, lptr.data(), size_t(N + 1) * 4));
  HIP_TRY(c, up(p.node_lterm, lterm.data(), lterm.size() * 4));
  HIP_TRY(c, up(p.node_nptr, nptr.data(), size_t(N + 1) * 4));
  HIP_TRY(c, up(p.node_nterm, nterm.data(), nterm.size() * 4));
  HIP_TRY(c, up(p.deg, deg.data(), size_t(N) * 8));
  std::vector<double> inv_deg(N), hinv_sus(L);
  for (int v = 0; v < N; ++v) inv_deg[v] = 1.0 / deg[v];
  for (int l = 0; l < L; ++l) hinv_sus[l] = 0.5 / sus[l];
  HIP_TRY(c, up(p.inv_deg, inv_deg.data(), size_t(N) * 8));
  HIP_TRY(c, up(p.hinv_sus, hinv_sus.data(), size_t(L) * 8));
  if (tiles_ok) {
    HIP_TRY(c, up(p.clus_n0, clus_n0.data(), clus_n0.size() * 4));
    HIP_TRY(c, up(p.tl_ptr, tl_ptr.data(), tl_ptr.size() * 4));
    HIP_TRY(c, up(p.tl, tl.data(), tl.size() * 4));
    HIP_TRY(c, up(p.tcsr, tcsr.data(), tcsr.size() * 4));
  }
  HIP_TRY(c, up(p.nc_node, nc_node.data(), size_t(Jnc) * 4));
  HIP_TRY(c, up(p.ramp_idx, ramp_idx.data(), size_t(G) * 4));
  HIP_TRY(c, up(p.gen_c2, n->gen_c2, size_t(G) * 8));
  HIP_TRY(c, up(p.gen_c1, n->gen_c1, size_t(G) * 8));
  HIP_TRY(c, up(p.gen_pmin, n->gen_pmin, size_t(G) * T * 8));
  HIP_TRY(c, up(p.gen_pmax, n->gen_pmax, size_t(G) * T * 8));
  HIP_TRY(c, up(p.gen_ramp, n->gen_ramp, size_t(G) * 8));
  HIP_TRY(c, up(p.load_d, n->load_d, size_t(D) * T * 8));
  HIP_TRY(c, up(p.bat_P, n->bat_P, size_t(B) * 8));
  HIP_TRY(c, up(p.bat_dur, n->bat_dur, size_t(B) * 8));
  HIP_TRY(c, up(p.bat_eta, n->bat_eta, size_t(B) * 8));
  HIP_TRY(c, up(p.bat_alpha, n->bat_alpha, size_t(B) * 8));
  // synchronise before the host vectors go out of scope
  HIP_TRY(c, hipStreamSynchronize(c->stream));

  Topo& tp = s.topo;
  tp.N = N; tp.T = T; tp.K = s.K; tp.Kp = s.Kp; tp.Kpp = Kpp; tp.L = L; tp.G = G;
  tp.D = D; tp.B = B; tp.Jnc = Jnc; tp.nR = s.nR;
  tp.line_from = reinterpret_cast<const int32_t*>(ws + p.line_from);
  tp.line_to = reinterpret_cast<const int32_t*>(ws + p.line_to);
  tp.sus = reinterpret_cast<const double*>(ws + p.sus);
  tp.cap = reinterpret_cast<const double*>(ws + p.cap);
  tp.outage_k = reinterpret_cast<const int32_t*>(ws + p.outage_k);
  tp.node_lptr = reinterpret_cast<const int32_t*>(ws + p.node_lptr);
  tp.node_lterm = reinterpret_cast<const int2*>(ws + p.node_lterm);
  tp.node_nptr = reinterpret_cast<const int32_t*>(ws + p.node_nptr);
  tp.node_nterm = reinterpret_cast<const int32_t*>(ws + p.node_nterm);
  tp.deg = reinterpret_cast<const double*>(ws + p.deg);
  tp.inv_deg = reinterpret_cast<const double*>(ws + p.inv_deg);
  tp.hinv_sus = reinterpret_cast<const double*>(ws + p.hinv_sus);
  tp.clus_n0 = reinterpret_cast<const int32_t*>(ws + p.clus_n0);
  tp.tl_ptr = reinterpret_cast<const int32_t*>(ws + p.tl_ptr);
  tp.tl = reinterpret_cast<const int4*>(ws + p.tl);
  tp.tcsr = reinterpret_cast<const int32_t*>(ws + p.tcsr);
  tp.Ldc = s.Ldc;
  tp.line_dc = reinterpret_cast<const int32_t*>(ws + p.line_dc);  // all -1 without DC links
  tp.n_chg = s.n_chg;
  tp.Zc = s.Zc;
  tp.chg_ptr = reinterpret_cast<const int32_t*>(ws + p.chg_ptr);
  tp.chg = reinterpret_cast<const LineChg*>(ws + p.chg);
  tp.nc_node = reinterpret_cast<const int32_t*>(ws + p.nc_node);
  tp.ramp_idx = reinterpret_cast<const int32_t*>(ws + p.ramp_idx);
  tp.gen_c2 = reinterpret_cast<const double*>(ws + p.gen_c2);
  tp.gen_c1 = reinterpret_cast<const double*>(ws + p.gen_c1);
  tp.gen_pmin = reinterpret_cast<const double*>(ws + p.gen_pmin);
  tp.gen_pmax = reinterpret_cast<const double*>(ws + p.gen_pmax);
  tp.gen_ramp = reinterpret_cast<const double*>(ws + p.gen_ramp);
  tp.load_d = reinterpret_cast<const double*>(ws + p.load_d);
  tp.bat_P = reinterpret_cast<const double*>(ws + p.bat_P);
  tp.bat_dur = reinterpret_cast<const double*>(ws + p.bat_dur);
  tp.bat_eta = reinterpret_cast<const double*>(ws + p.bat_eta);
  tp.bat_alpha = reinterpret_cast<const double*>(ws + p.bat_alpha);

  s.ctl = reinterpret_cast<Ctl*>(ws + p.ctl);
  s.ring = reinterpret_cast<Rec*>(ws + p.ring);
  for (Geom* g : {&s.geom64, &s.geom32}) {
    g->part_sweep = reinterpret_cast<double*>(ws + p.part_sweep);
    g->part_nc = reinterpret_cast<double*>(ws + p.part_nc);
    g->ctl = s.ctl;
    g->ring = s.ring;
  }
  const bool has32 = c->opt.state_dtype == OPF_F32;
  const bool has64 = !has32 || c->opt.polish_fp64;
  s.state_begin = SIZE_MAX;
  s.state_end = 0;
  if (has64) {
    s.st64 = state_ptrs<double, double>(ws, p.o64);
    s.state_begin = std::min(s.state_begin, p.o64.begin);
    s.state_end = std::max(s.state_end, p.o64.end);
  }
  if (has32) {
    if (c->bf16_duals)
      s.st32b = state_ptrs<float, bf16_t>(ws, p.o32);
    else
      s.st32 = state_ptrs<float, float>(ws, p.o32);
    s.state_begin = std::min(s.state_begin, p.o32.begin);
    s.state_end = std::max(s.state_end, p.o32.end);
  }
  s.eps_eff = c->opt.eps * (c->opt.eps_relative ? load_rms : 1.0);
  const double J = 2.0 * L + Jnc;
  s.rms_norm = std::sqrt(2.0 * J * T * double(s.Kp));
  return OPF_OK;
}

opf_status load(opf_ctx* c, const opf_network* nets, int count, void* d_ws, size_t bytes) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!d_ws) return fail(c, OPF_E_INVALID, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign)
    return fail(c, OPF_E_INVALID, "workspace must be 256-byte aligned");
  std::vector<Inst> insts;
  std::vector<InstPlan> plans;
  std::vector<Tables> tabs;
  BatchPlan bp{};
  Layout lay;
  opf_status s = plan_all(c, nets, count, insts, plans, bp, lay, &tabs);
  if (s != OPF_OK) return s;
  if (bytes < lay.total)
    return fail(c, OPF_E_OOM, "workspace too small: need " + std::to_string(lay.total) + " bytes");
  if (c->h_ctl_count < count) {
    if (c->h_ctl) (void)hipHostFree(c->h_ctl);
    c->h_ctl = nullptr;
    c->h_ctl_count = 0;
    HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_ctl), sizeof(Ctl) * count));
    c->h_ctl_count = count;
  }
  if (!c->h_rec) HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_rec), sizeof(Rec) * kRing));
  if (!c->h_int) HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_int), 64));
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->loaded = false;
  c->ws = static_cast<char*>(d_ws);
  c->ws_bytes = bytes;
  c->batch = count > 1;
  // a batch's work items default to four period groups (each handed out as
  // a workgroup frees up; measured best on the uneven 64-instance batch),
  // one instance's to one; opf_autotune picks from 1, 2, 4, 8
  c->tile_groups = c->batch ? 4 : 1;
  HIP_TRY(c, hipMemsetAsync(c->ws, 0, lay.total, c->stream));
  c->max_T = 1;
  for (int i = 0; i < count; ++i) {
    s = upload_instance(c, &nets[i], insts[i], plans[i], tabs[i]);
    if (s != OPF_OK) return s;
    c->max_T = std::max(c->max_T, insts[i].T);
  }
  c->inst = std::move(insts);
  c->has32 = c->opt.state_dtype == OPF_F32;
  c->has64 = !c->has32 || c->opt.polish_fp64;
  if (c->batch) {
    c->d_descs64 = c->ws + bp.descs64;
    c->d_descs32 = c->ws + bp.descs32;
    c->d_dev_prefix = reinterpret_cast<int64_t*>(c->ws + bp.dev_prefix);
    c->d_grp64 = reinterpret_cast<int64_t*>(c->ws + bp.grp64);
    c->d_grp32 = reinterpret_cast<int64_t*>(c->ws + bp.grp32);
    c->d_tiles64 = reinterpret_cast<int64_t*>(c->ws + bp.tiles64);
    c->d_tiles32 = reinterpret_cast<int64_t*>(c->ws + bp.tiles32);
    c->d_queue = reinterpret_cast<int32_t*>(c->ws + bp.queue);
  }
  s = refresh_geometry(c);
  if (s != OPF_OK) return s;
  s = reset_state(c);
  if (s != OPF_OK) return s;
  c->tape = TapePlan{};
  c->tape_hist.clear();
  c->loaded = true;
  return OPF_OK;
}

opf_status check_inst(opf_ctx* c, int32_t i) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!c->loaded) return fail(c, OPF_E_STATE, not_loaded_msg(c));
  if (i < 0 || i >= int(c->inst.size())) return fail(c, OPF_E_INVALID, "instance out of range");
  return OPF_OK;
}

// Enqueues one block of iterations for the solve loop, as a captured graph
// where possible.
opf_status enqueue_block(opf_ctx* c, int blk, bool graph_ok) {
  const int ae = c->opt.adapt_every;
  const bool aligned = ae == 0 || c->host_iter % ae == 0;
  if (graph_ok && aligned) {
    const auto key = std::make_pair(c->precision, blk);
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
      hipGraph_t gr;
      HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      enqueue_n(c, blk, true, 0);
      HIP_TRY(c, hipStreamEndCapture(c->stream, &gr));
      hipGraphExec_t ex;
      HIP_TRY(c, hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
      (void)hipGraphDestroy(gr);
      it = c->graphs.emplace(key, ex).first;
    }
    HIP_TRY(c, hipGraphLaunch(it->second, c->stream));
    c->host_iter += blk;
  } else {
    const int n = (graph_ok && !aligned) ? int(ae - c->host_iter % ae) : blk;
    enqueue_n(c, n, false, c->host_iter);
    c->host_iter += n;
  }
  HIP_TRY(c, hipGetLastError());
  return OPF_OK;
}

bool all_done(const opf_ctx* c) {
  for (size_t i = 0; i < c->inst.size(); ++i)
    if (!c->h_ctl[i].done) return false;
  return true;
}

// ---------------------------------------------------------------------------
// Tape of a forward run and its adjoint.

size_t elem_size(int precision) { return precision == 0 ? sizeof(double) : sizeof(float); }

SnapLayout snap_layout(const Inst& s, int precision) {
  const size_t S = elem_size(precision);
  const size_t line = size_t(s.L) * s.T * s.Kpp * S, node = size_t(s.N) * s.T * s.Kpp * S;
  const size_t sizes[kSnapArrays] = {
      line, line, line, line, size_t(s.T) * s.Kpp * S, node, node, node,
      size_t(s.N) * s.T * S, size_t(s.N) * s.T * S, size_t(s.Jnc) * s.T * S,
      size_t(s.Jnc) * s.T * S, size_t(s.Jnc) * s.T * S, 4 * size_t(s.nR) * s.T * S,
      6 * size_t(s.B) * s.T * S, size_t(s.Ldc) * s.T * s.Kpp * S, size_t(s.Zc) * s.T * S};
  SnapLayout sl{};
  Layout L;
  for (int i = 0; i < kSnapArrays; ++i) {
    sl.bytes[i] = sizes[i];
    sl.off[i] = L.take(sizes[i]);
  }
  sl.total = L.total;
  return sl;
}

TapePlan plan_tape(const Inst& s, int precision, int M, int C) {
  TapePlan t;
  t.n_iters = M;
  t.every = C;
  t.precision = precision;
  t.snap = snap_layout(s, precision);
  const size_t S = elem_size(precision);
  Layout L;
  t.hist = L.take(sizeof(Ctl) * (size_t(M) + 1));
  t.n_ckpt = (size_t(M) + C - 1) / C;
  t.ckpt = L.take(t.snap.total * t.n_ckpt);
  t.final_snap = L.take(t.snap.total);
  t.seg = L.take(t.snap.total * size_t(C - 1));  // a segment's iterates after its checkpoint
  t.mask_words = mask_words(s.nR, s.B, (s.T + kWave - 1) / kWave);
  t.masks = L.take(t.mask_words * sizeof(uint32_t) * size_t(M));
  t.adj_begin = L.total;
  const size_t line = size_t(s.L) * s.T * s.Kpp * S, node = size_t(s.N) * s.T * s.Kpp * S;
  for (int b = 0; b < 2; ++b) {
    for (int q = 0; q < 4; ++q) t.adj_line[b][q] = L.take(line);
    t.adj_td[b] = L.take(size_t(s.T) * s.Kpp * S);
    t.adj_hd[b] = L.take(size_t(s.Ldc) * s.T * s.Kpp * S);
    t.adj_tz[b] = L.take(size_t(s.Zc) * s.T * S);
    for (int q = 0; q < 3; ++q) t.adj_node[b][q] = L.take(node);
  }
  const size_t nt = size_t(s.N) * s.T * S, jt = size_t(s.Jnc) * s.T * S;
  t.gsp = L.take(nt);
  t.gsb = L.take(nt);
  for (int q = 0; q < 5; ++q) t.dev[q] = L.take(jt);
  t.ramp_adj = L.take(4 * size_t(s.nR) * s.T * S);
  t.bat_adj = L.take(6 * size_t(s.B) * s.T * S);
  t.gcap = L.take(size_t(s.L) * s.T * s.Kpp * sizeof(double));
  t.gload = L.take(size_t(s.D) * s.T * sizeof(double));
  t.gpmax = L.take(size_t(s.G) * s.T * sizeof(double));
  t.adj_end = L.total;
  t.total = L.total;
  return t;
}

// Device arrays of the iterate (buffer cur) in snapshot order.
template <typename R>
void state_arrays(const State<R, R>& st, int cur, char* (&out)[kSnapArrays]) {
  const Buf<R, R>& b = st.buf[cur];
  char* a[kSnapArrays] = {
      reinterpret_cast<char*>(b.P), reinterpret_cast<char*>(b.Tm), reinterpret_cast<char*>(b.V1),
      reinterpret_cast<char*>(b.V2), reinterpret_cast<char*>(b.Td), reinterpret_cast<char*>(b.U),
      reinterpret_cast<char*>(b.W), reinterpret_cast<char*>(b.TB),
      reinterpret_cast<char*>(st.avgW), reinterpret_cast<char*>(st.avgTB),
      reinterpret_cast<char*>(st.pnc), reinterpret_cast<char*>(st.thnc),
      reinterpret_cast<char*>(st.vbar), reinterpret_cast<char*>(st.ramp_st),
      reinterpret_cast<char*>(st.bat_st), reinterpret_cast<char*>(b.Hd),
      reinterpret_cast<char*>(b.Tz)};
  for (int i = 0; i < kSnapArrays; ++i) out[i] = a[i];
}

template <typename R>
const State<R, R>& inst_state(const Inst& s);
template <>
const State<double, double>& inst_state<double>(const Inst& s) {
  return s.st64;
}
template <>
const State<float, float>& inst_state<float>(const Inst& s) {
  return s.st32;
}

// Copies the iterate (buffer cur) into the snapshot at snap, or back; with
// ctl_to, the same launch also copies the control block there.
template <typename R>
void snapshot(opf_ctx* c, const Inst& s, int cur, char* snap, bool to_snap,
              Ctl* ctl_to = nullptr) {
  char* arr[kSnapArrays];
  state_arrays<R>(inst_state<R>(s), cur, arr);
  CopyList cl{};
  const SnapLayout& sl = c->tape.snap;
  for (int i = 0; i < kSnapArrays; ++i) {
    if (sl.bytes[i] == 0) continue;
    cl.src[cl.n] = to_snap ? arr[i] : snap + sl.off[i];
    cl.dst[cl.n] = to_snap ? snap + sl.off[i] : arr[i];
    cl.bytes[cl.n] = sl.bytes[i];
    ++cl.n;
  }
  if (ctl_to) {
    cl.src[cl.n] = reinterpret_cast<const char*>(s.ctl);
    cl.dst[cl.n] = reinterpret_cast<char*>(ctl_to);
    cl.bytes[cl.n] = sizeof(Ctl);
    ++cl.n;
  }
  launch_copy(cl, c->stream);
}

char* tape_ptr(const opf_ctx* c, size_t off) { return c->tape.base + off; }

// Adjoint kernel arguments for the reverse of iteration i from the snapshot
// at snap; ob selects which adjoint buffer holds the adjoint after it.
template <typename R>
AdjArgs<R> adj_args(opf_ctx* c, const Inst& s, const char* snap, int ob, double w_obj) {
  const TapePlan& t = c->tape;
  const SnapLayout& sl = t.snap;
  AdjArgs<R> a{};
  a.tp = s.topo;
  auto sp = [&](int i) { return reinterpret_cast<R*>(const_cast<char*>(snap) + sl.off[i]); };
  a.A.P = sp(0);
  a.A.Tm = sp(1);
  a.A.V1 = sp(2);
  a.A.V2 = sp(3);
  a.A.Td = sp(4);
  a.A.Hd = sp(15);
  a.A.Tz = sp(16);
  a.A.U = sp(5);
  a.A.W = sp(6);
  a.A.TB = sp(7);
  a.avgW = sp(8);
  a.avgTB = sp(9);
  a.pnc = sp(10);
  a.thnc = sp(11);
  a.vbar = sp(12);
  a.ramp_st = sp(13);
  a.bat_st = sp(14);
  auto tp = [&](size_t off) { return reinterpret_cast<R*>(tape_ptr(c, off)); };
  for (int side = 0; side < 2; ++side) {
    const int b = side == 0 ? ob : ob ^ 1;
    AdjBuf<R>& d = side == 0 ? a.out : a.in;
    d.P = tp(t.adj_line[b][0]);
    d.Tm = tp(t.adj_line[b][1]);
    d.V1 = tp(t.adj_line[b][2]);
    d.V2 = tp(t.adj_line[b][3]);
    d.Td = tp(t.adj_td[b]);
    d.Hd = tp(t.adj_hd[b]);
    d.Tz = tp(t.adj_tz[b]);
    d.U = tp(t.adj_node[b][0]);
    d.W = tp(t.adj_node[b][1]);
    d.TB = tp(t.adj_node[b][2]);
  }
  a.gsp = tp(t.gsp);
  a.gsb = tp(t.gsb);
  a.dev_p = tp(t.dev[0]);
  a.dev_th = tp(t.dev[1]);
  a.dev_v = tp(t.dev[2]);
  a.dev_x = tp(t.dev[3]);
  a.dev_t = tp(t.dev[4]);
  a.ramp_adj = tp(t.ramp_adj);
  a.bat_adj = tp(t.bat_adj);
  a.gcap = reinterpret_cast<double*>(tape_ptr(c, t.gcap));
  a.gload = reinterpret_cast<double*>(tape_ptr(c, t.gload));
  a.gpmax = reinterpret_cast<double*>(tape_ptr(c, t.gpmax));
  const Geom& g = t.precision == 0 ? s.geom64 : s.geom32;
  a.nv = g.nv;
  a.lanes_per_row = g.lanes_per_row;
  a.n_grps = g.n_grps;
  a.inner_iters = g.inner_iters;
  a.omega_scale = g.omega_scale;
  a.w_obj = w_obj;
  return a;
}

opf_status tape_check(opf_ctx* c) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!c->loaded) return fail(c, OPF_E_STATE, not_loaded_msg(c));
  if (c->batch) return fail(c, OPF_E_INVALID, "the adjoint supports one instance, not a batch");
  if (c->bf16_duals) return fail(c, OPF_E_INVALID, "the adjoint needs FP32 or FP64 duals, not BF16");
  if (c->opt.inner_iters > kMaxAdjInner)
    return fail(c, OPF_E_INVALID, "the adjoint supports inner_iters <= 32");
  return OPF_OK;
}

// After a recorded run the control block holds the run's own iteration
// limits; later opf_iterate / opf_solve calls use the configured ones again.
opf_status restore_limits(opf_ctx* c) {
  opf_status s = read_ctls(c);
  if (s != OPF_OK) return s;
  Ctl& h = c->h_ctl[0];
  h.min_iter = c->opt.min_iter;
  h.max_iter = c->opt.max_iter;
  h.done = (h.converged || h.numeric_bad || h.iter >= h.max_iter) ? 1 : 0;
  HIP_TRY(c, hipMemcpyAsync(c->inst[0].ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return OPF_OK;
}

// Records a forward run.  From the zero start (warm = false): exactly M
// iterations.  From the current iterate (warm = true): the stopping rule of
// the options after at least min_iters and at most M iterations.  The
// iterations actually run become the tape.
template <typename R>
opf_status tape_forward(opf_ctx* c, int M, int C, bool warm, int min_iters, int* n_run) {
  const Inst& s = c->inst[0];
  TapePlan& t = c->tape;
  opf_status st = OPF_OK;
  if (!warm) {
    st = reset_state(c);
    if (st != OPF_OK) return st;
  }
  st = read_ctls(c);
  if (st != OPF_OK) return st;
  Ctl& h0 = c->h_ctl[0];
  const int iter0 = h0.iter, cur0 = h0.cur;
  if (warm) {
    h0.min_iter = iter0 + min_iters;
    h0.max_iter = iter0 + M;
    h0.done = 0;
    h0.converged = 0;
  } else {  // exactly M iterations
    h0.min_iter = INT32_MAX;
    h0.max_iter = INT32_MAX;
  }
  HIP_TRY(c, hipMemcpyAsync(s.ctl, &h0, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  Ctl* hist = reinterpret_cast<Ctl*>(tape_ptr(c, t.hist));
  Geom& geo = c->tape.precision == 0 ? c->inst[0].geom64 : c->inst[0].geom32;
  struct MaskOff {  // later iterations record nothing, however this returns
    Geom& g;
    ~MaskOff() { g.mask_rec = nullptr; }
  } mask_off{geo};
  for (int i = 0; i < M; ++i) {
    geo.mask_rec = reinterpret_cast<uint32_t*>(
        tape_ptr(c, t.masks + sizeof(uint32_t) * t.mask_words * size_t(i)));
    if (i % C == 0)  // the checkpoint and the control block in one copy launch
      snapshot<R>(c, s, (cur0 + i) & 1, tape_ptr(c, t.ckpt + t.snap.total * (i / C)), true,
                  hist + i);
    else
      HIP_TRY(c, hipMemcpyAsync(hist + i, s.ctl, sizeof(Ctl), hipMemcpyDeviceToDevice,
                                c->stream));
    enqueue_n(c, 1, false, int64_t(iter0) + i);
  }
  geo.mask_rec = nullptr;
  HIP_TRY(c, hipMemcpyAsync(hist + M, s.ctl, sizeof(Ctl), hipMemcpyDeviceToDevice, c->stream));
  c->tape_hist.assign(size_t(M) + 1, Ctl{});
  HIP_TRY(c, hipMemcpyAsync(c->tape_hist.data(), hist, sizeof(Ctl) * (size_t(M) + 1),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int ran = c->tape_hist[M].iter - iter0;  // iterations before the stop
  if (ran < 0 || ran > M) return fail(c, OPF_E_STATE, "forward run lost its iteration count");
  for (int i = 0; i <= ran; ++i) {
    const Ctl& h = c->tape_hist[i];
    if (h.numeric_bad) return fail(c, OPF_E_NUMERIC, "residual became NaN or infinite");
    if (h.iter != iter0 + i || h.cur != ((cur0 + i) & 1))
      return fail(c, OPF_E_STATE, "forward run did not advance one iteration per step");
  }
  c->tape_hist.resize(size_t(ran) + 1);
  snapshot<R>(c, s, c->tape_hist[ran].cur, tape_ptr(c, t.final_snap), true);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  t.n_iters = ran;
  t.n_ckpt = (size_t(ran) + C - 1) / C;
  c->host_iter = c->tape_hist[ran].iter;
  t.ready = true;
  if (n_run) *n_run = ran;
  return restore_limits(c);
}

template <typename R>
opf_status adjoint(opf_ctx* c, const double* cot, double w_obj, double* grad_load,
                   double* grad_cap, double* grad_pmax) {
  const Inst& s = c->inst[0];
  TapePlan& t = c->tape;
  const int M = t.n_iters, C = t.every;
  HIP_TRY(c, hipMemsetAsync(tape_ptr(c, t.adj_begin), 0, t.adj_end - t.adj_begin, c->stream));
  int ob = 0;
  {
    AdjArgs<R> a = adj_args<R>(c, s, tape_ptr(c, t.final_snap), ob, w_obj);
    launch_adj_init<R>(a, cot, c->stream);
  }
  Ctl* hist = reinterpret_cast<Ctl*>(tape_ptr(c, t.hist));
  for (int seg = int(t.n_ckpt) - 1; seg >= 0; --seg) {
    const int i0 = seg * C, i1 = std::min(M, i0 + C);
    char* ck = tape_ptr(c, t.ckpt + t.snap.total * seg);
    // the segment's later iterates, recomputed from its checkpoint (the
    // reverse reads the first one from the checkpoint itself)
    auto iterate_at = [&](int i) {
      return i == i0 ? ck : tape_ptr(c, t.seg + t.snap.total * (i - i0 - 1));
    };
    if (i1 - i0 > 1) {
      snapshot<R>(c, s, c->tape_hist[i0].cur, ck, false);
      HIP_TRY(c, hipMemcpyAsync(s.ctl, hist + i0, sizeof(Ctl), hipMemcpyDeviceToDevice,
                                c->stream));
      for (int i = i0; i + 1 < i1; ++i) {
        enqueue_n(c, 1, false, c->tape_hist[i].iter);
        snapshot<R>(c, s, c->tape_hist[i + 1].cur, iterate_at(i + 1), true);
      }
    }
    for (int i = i1 - 1; i >= i0; --i) {
      AdjArgs<R> a = adj_args<R>(c, s, iterate_at(i), ob, w_obj);
      a.masks = reinterpret_cast<const uint32_t*>(
          tape_ptr(c, t.masks + sizeof(uint32_t) * t.mask_words * size_t(i)));
      const Ctl& h = c->tape_hist[i];
      a.s.rp = h.rho_p;
      a.s.rt = h.rho_th;
      a.s.su = h.su;
      a.s.sv = h.sv;
      a.s.su_next = c->tape_hist[i + 1].su;
      a.s.last = i == M - 1;
      launch_adj_iteration<R>(a, c->stream);
      ob ^= 1;
    }
    HIP_TRY(c, hipGetLastError());
  }
  AdjArgs<R> a = adj_args<R>(c, s, tape_ptr(c, t.final_snap), ob, w_obj);
  if (grad_cap) launch_adj_cap<R>(a, grad_cap, c->stream);
  if (grad_load && s.D > 0)
    HIP_TRY(c, hipMemcpyAsync(grad_load, a.gload, sizeof(double) * s.D * s.T,
                              hipMemcpyDeviceToDevice, c->stream));
  if (grad_pmax && s.G > 0)
    HIP_TRY(c, hipMemcpyAsync(grad_pmax, a.gpmax, sizeof(double) * s.G * s.T,
                              hipMemcpyDeviceToDevice, c->stream));
  // leave the iterate where the forward run left it
  snapshot<R>(c, s, c->tape_hist[M].cur, tape_ptr(c, t.final_snap), false);
  HIP_TRY(c, hipMemcpyAsync(s.ctl, hist + M, sizeof(Ctl), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->host_iter = c->tape_hist[M].iter;
  return restore_limits(c);
}

// ---------------------------------------------------------------------------
// Iterate export/import (warm start) and layout queries.

struct BlobHead {
  char magic[8];
  int32_t version, precision, N, T, K, L, Jnc, nR, B;
  double rho_p, rho_th;
  double su, sv;  // pending rescale ratios (deferred to the next iteration)
  int32_t Ldc, n_chg, Zc;
  uint64_t topo_hash;
};
constexpr size_t kBlobHead = 256;
static_assert(sizeof(BlobHead) <= kBlobHead, "blob header");

template <typename R>
opf_status state_copy(opf_ctx* c, const Inst& s, int cur, char* blob, bool to_blob,
                      const SnapLayout& sl) {
  char* arr[kSnapArrays];
  state_arrays<R>(inst_state<R>(s), cur, arr);
  for (int i = 0; i < kSnapArrays; ++i) {
    if (sl.bytes[i] == 0) continue;
    char* b = blob + kBlobHead + sl.off[i];
    HIP_TRY(c, hipMemcpyAsync(to_blob ? b : arr[i], to_blob ? arr[i] : b, sl.bytes[i],
                              hipMemcpyDefault, c->stream));
  }
  return OPF_OK;
}

// Forgets this context's hold on its device's fixed workspace (a load into
// a caller workspace, or destroy).
void release_static(opf_ctx* c) {
  if (c && c->static_dev >= 0) {
    static_workspace_release(c->static_dev, c);
    c->static_dev = -1;
  }
}

opf_status state_check(opf_ctx* c) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!c->loaded) return fail(c, OPF_E_STATE, not_loaded_msg(c));
  if (c->batch) return fail(c, OPF_E_INVALID, "state export/import is per single instance");
  if (c->bf16_duals) return fail(c, OPF_E_INVALID, "state export/import needs FP32 or FP64 duals");
  return OPF_OK;
}

}  // namespace

extern "C" {

void opf_default_options(opf_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->state_dtype = OPF_F64;
  o->dual_dtype = OPF_F64;
  o->rho_p = 1.0;
  o->rho_theta = 1.0;
  o->mu = 2.0;
  o->gamma = 1.1;
  o->adapt_every = 10;
  o->eps = 1e-3;
  o->eps_relative = 1;
  o->max_iter = 10000;
  o->min_iter = 0;
  o->block_iters = 50;
  o->check_every = 1;
  o->inner_iters = 10;
  o->inner_omega_scale = 1.0;
  o->polish_fp64 = 1;
  o->polish_factor = 1.2;
  o->use_graphs = 1;
  o->hip_stream = nullptr;
  o->sweep_tiles = -1;
}

opf_status opf_create(const opf_options* opt, opf_ctx** out) {
  if (!out) return fail(nullptr, OPF_E_INVALID, "out is NULL");
  *out = nullptr;
  opf_options o;
  if (opt)
    o = *opt;
  else
    opf_default_options(&o);
  if (o.state_dtype != OPF_F64 && o.state_dtype != OPF_F32)
    return fail(nullptr, OPF_E_INVALID, "state_dtype must be OPF_F64 or OPF_F32");
  if (o.dual_dtype != o.state_dtype && !(o.state_dtype == OPF_F32 && o.dual_dtype == OPF_BF16))
    return fail(nullptr, OPF_E_INVALID, "dual_dtype must equal state_dtype or be BF16 with F32");
  if (!(o.rho_p > 0) || !(o.rho_theta > 0) || !std::isfinite(o.rho_p) || !std::isfinite(o.rho_theta))
    return fail(nullptr, OPF_E_INVALID, "penalties must be finite and > 0");
  if (!(o.mu >= 1.0) || !(o.gamma >= 1.0)) return fail(nullptr, OPF_E_INVALID, "need mu >= 1, gamma >= 1");
  if (o.adapt_every < 0 || o.check_every < 1 || (o.adapt_every > 0 && o.adapt_every % o.check_every))
    return fail(nullptr, OPF_E_INVALID, "need adapt_every >= 0, check_every >= 1 dividing adapt_every");
  if (!(o.eps >= 0.0)) return fail(nullptr, OPF_E_INVALID, "eps must be >= 0");
  if (o.max_iter < 0 || o.min_iter < 0 || o.block_iters < 1)
    return fail(nullptr, OPF_E_INVALID, "need max_iter >= 0, min_iter >= 0, block_iters >= 1");
  if (!(o.polish_factor >= 1.0)) return fail(nullptr, OPF_E_INVALID, "polish_factor must be >= 1");
  if (o.sweep_tiles < -1 || o.sweep_tiles > 1)
    return fail(nullptr, OPF_E_INVALID, "sweep_tiles must be -1, 0 or 1");
  if (o.inner_iters < 1 || !(o.inner_omega_scale > 0))
    return fail(nullptr, OPF_E_INVALID, "need inner_iters >= 1 and inner_omega_scale > 0");
  opf_ctx* c = new opf_ctx();
  c->opt = o;
  c->stream = reinterpret_cast<hipStream_t>(o.hip_stream);
  c->bf16_duals = o.dual_dtype == OPF_BF16;
  c->tile_mode = o.sweep_tiles;
  // set-up that later calls rely on to allocate nothing: the pinned readback
  // buffers of one instance, and the device address of this device's fixed
  // workspace.  Without a usable GPU both are left for later (the host-only
  // calls, e.g. opf_workspace_size, still work).
  int dev = -1;
  if (hipGetDevice(&dev) == hipSuccess) {
    (void)static_workspace_setup(dev);
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_ctl), sizeof(Ctl)) == hipSuccess)
      c->h_ctl_count = 1;
    else
      c->h_ctl = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_rec), sizeof(Rec) * kRing) != hipSuccess)
      c->h_rec = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_int), 64) != hipSuccess) c->h_int = nullptr;
  }
  (void)hipGetLastError();
  *out = c;
  return OPF_OK;
}

opf_status opf_check_network(const opf_network* n, const opf_options* opt, int32_t* tiled) {
  opf_ctx tmp;  // host only: no stream, no device memory
  if (opt)
    tmp.opt = *opt;
  else
    opf_default_options(&tmp.opt);
  std::vector<Inst> insts;
  std::vector<InstPlan> plans;
  std::vector<Tables> tabs;
  BatchPlan bp{};
  Layout lay;
  const opf_status s = plan_all(&tmp, n, 1, insts, plans, bp, lay, &tabs);
  if (s != OPF_OK) {
    g_create_error = tmp.err;
    return s;
  }
  if (tiled) *tiled = tabs[0].tiles_ok ? 1 : 0;
  return OPF_OK;
}

opf_status opf_workspace_size(opf_ctx* c, const opf_network* n, size_t* bytes) {
  return workspace_size(c, n, 1, bytes);
}

opf_status opf_workspace_size_batch(opf_ctx* c, const opf_network* nets, int32_t count,
                                    size_t* bytes) {
  return workspace_size(c, nets, count, bytes);
}

opf_status opf_load_network(opf_ctx* c, const opf_network* n, void* d_ws, size_t bytes) {
  release_static(c);
  return load(c, n, 1, d_ws, bytes);
}

opf_status opf_load_batch(opf_ctx* c, const opf_network* nets, int32_t count, void* d_ws,
                          size_t bytes) {
  release_static(c);
  return load(c, nets, count, d_ws, bytes);
}

opf_status opf_load_network_static(opf_ctx* c, const opf_network* n) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  int dev = -1;
  HIP_TRY(c, hipGetDevice(&dev));
  // the device address of this device's array (taken once, at opf_create or
  // on the first call on the device)
  HIP_TRY(c, static_workspace_setup(dev));
  void* ws = static_workspace(dev);
  if (!ws) return fail(c, OPF_E_HIP, "no device address for the fixed workspace");
  if (!c->h_ctl || c->h_ctl_count < 1 || !c->h_rec || !c->h_int)
    return fail(c, OPF_E_STATE, "the context's pinned readback buffers are missing (opf_create "
                                "ran without a usable GPU)");
  size_t need = 0;
  opf_status st = workspace_size(c, n, 1, &need);
  if (st != OPF_OK) return st;
  if (need > kStaticWorkspaceBytes)
    return fail(c, OPF_E_OOM, "network needs a " + std::to_string(need) +
                                  "-byte workspace; the fixed workspace holds " +
                                  std::to_string(kStaticWorkspaceBytes) + " bytes");
  const void* prev = static_workspace_claim(dev, c);
  if (prev && prev != c) {
    // the previous holder's work is finished before its iterate is replaced;
    // it can no longer be used until it loads again
    opf_ctx* p = const_cast<opf_ctx*>(static_cast<const opf_ctx*>(prev));
    (void)hipStreamSynchronize(p->stream);
    p->loaded = false;
    p->taken_over = true;
    p->static_dev = -1;
  }
  c->static_dev = dev;
  c->taken_over = false;
  return load(c, n, 1, ws, kStaticWorkspaceBytes);
}

opf_status opf_num_instances(opf_ctx* c, int32_t* count) {
  if (!c || !count) return fail(c, OPF_E_INVALID, "NULL argument");
  *count = c->loaded ? int32_t(c->inst.size()) : 0;
  return OPF_OK;
}

opf_status opf_reset(opf_ctx* c) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!c->loaded) return fail(c, OPF_E_STATE, not_loaded_msg(c));
  return reset_state(c);
}

opf_status opf_iterate(opf_ctx* c, int32_t n) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!c->loaded) return fail(c, OPF_E_STATE, not_loaded_msg(c));
  if (n < 0) return fail(c, OPF_E_INVALID, "n_iters must be >= 0");
  enqueue_n(c, n, false, c->host_iter);
  c->host_iter += n;
  HIP_TRY(c, hipGetLastError());
  return OPF_OK;
}

opf_status opf_solve(opf_ctx* c, opf_resid* out) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!c->loaded) return fail(c, OPF_E_STATE, not_loaded_msg(c));
  // Stopped batch instances leave the work lists at block boundaries, so
  // later blocks launch work only for those still running (their iterates
  // are untouched either way); the lists are whole again on return.
  struct Unretire {
    opf_ctx* c;
    ~Unretire() { (void)set_retired(c, {}); }
  } unretire{c};
  const int blk = c->opt.block_iters;
  const int ae = c->opt.adapt_every;
  // graphs need a capturable (non-null) stream and blocks aligned to the
  // penalty-update period
  const bool graph_ok = c->opt.use_graphs && !c->timing && c->stream != nullptr &&
                        (ae == 0 || blk % ae == 0);
  opf_status s = read_ctls(c);
  if (s != OPF_OK) return s;
  bool numeric = false;
  while (!all_done(c) && c->host_iter < int64_t(c->opt.max_iter)) {
    s = enqueue_block(c, blk, graph_ok);
    if (s != OPF_OK) return s;
    s = read_ctls(c);
    if (s != OPF_OK) return s;
    for (size_t i = 0; i < c->inst.size(); ++i) numeric = numeric || c->h_ctl[i].numeric_bad;
    if (numeric) break;
    if (c->batch) {
      std::vector<char> r(c->inst.size());
      for (size_t i = 0; i < r.size(); ++i) r[i] = c->h_ctl[i].done ? 1 : 0;
      s = set_retired(c, r);
      if (s != OPF_OK) return s;
    }
    // FP64 polish of a single FP32 instance near the tolerance
    if (!c->batch && c->precision == 1 && c->opt.polish_fp64 && c->has64 && !c->h_ctl[0].done) {
      opf_resid r;
      s = last_record(c, 0, &r);
      if (s != OPF_OK) return s;
      if (r.iter > 0 &&
          std::max(r.rms_primal, r.rms_dual) <= c->opt.polish_factor * c->inst[0].eps_eff) {
        s = widen_to_fp64(c);
        if (s != OPF_OK) return s;
      }
    }
  }
  s = read_ctls(c);
  if (s != OPF_OK) return s;
  opf_resid r;
  s = last_record(c, 0, &r);
  if (s != OPF_OK) return s;
  if (out) *out = r;
  if (numeric) return fail(c, OPF_E_NUMERIC, "residual became NaN or infinite");
  for (size_t i = 0; i < c->inst.size(); ++i)
    if (!c->h_ctl[i].converged) return OPF_NOT_CONVERGED;
  return OPF_OK;
}

opf_status opf_residuals_i(opf_ctx* c, int32_t i, opf_resid* out) {
  opf_status s = check_inst(c, i);
  if (s != OPF_OK) return s;
  if (!out) return fail(c, OPF_E_INVALID, "out is NULL");
  s = read_ctls(c);
  if (s != OPF_OK) return s;
  s = last_record(c, i, out);
  if (s != OPF_OK) return s;
  if (c->h_ctl[i].numeric_bad) return fail(c, OPF_E_NUMERIC, "residual became NaN or infinite");
  return OPF_OK;
}

opf_status opf_residuals(opf_ctx* c, opf_resid* out) { return opf_residuals_i(c, 0, out); }

opf_status opf_residual_history_i(opf_ctx* c, int32_t inst, opf_resid* out, int32_t max,
                                  int32_t* n) {
  opf_status s = check_inst(c, inst);
  if (s != OPF_OK) return s;
  if (!out || !n || max < 0) return fail(c, OPF_E_INVALID, "bad argument");
  s = read_ctls(c);
  if (s != OPF_OK) return s;
  const int iter = c->h_ctl[inst].iter;
  const int ce = std::max(1, c->opt.check_every);
  HIP_TRY(c, hipMemcpyAsync(c->h_rec, c->inst[inst].ring, sizeof(Rec) * kRing,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int first = std::max(1, iter - kRing + 1);
  int cnt = 0;
  for (int i = first; i <= iter && cnt < max; ++i) {
    if (i % ce) continue;
    const Rec& r = c->h_rec[(i - 1) % kRing];
    opf_resid& o = out[cnt++];
    std::memset(&o, 0, sizeof(o));
    fill_resid(r, &o);
    o.iter = r.iter;
  }
  *n = cnt;
  return OPF_OK;
}

opf_status opf_residual_history(opf_ctx* c, opf_resid* out, int32_t max, int32_t* n) {
  return opf_residual_history_i(c, 0, out, max, n);
}

opf_status opf_field_size_i(opf_ctx* c, int32_t inst, int32_t field, size_t* count) {
  opf_status s = check_inst(c, inst);
  if (s != OPF_OK) return s;
  if (!count) return fail(c, OPF_E_INVALID, "NULL argument");
  const Inst& x = c->inst[inst];
  const size_t KT = size_t(x.Kp) * x.T;
  if (field >= OPF_FIELD_P && field <= OPF_FIELD_V2)
    *count = KT * x.L;
  else if (field >= OPF_FIELD_U && field <= OPF_FIELD_THBAR)
    *count = KT * x.N;
  else if (field >= OPF_FIELD_PNC && field <= OPF_FIELD_VNC)
    *count = size_t(x.Jnc) * x.T;
  else
    return fail(c, OPF_E_INVALID, "unknown field");
  return OPF_OK;
}

opf_status opf_field_size(opf_ctx* c, int32_t field, size_t* count) {
  return opf_field_size_i(c, 0, field, count);
}

opf_status opf_get_field_i(opf_ctx* c, int32_t inst, int32_t field, double* dst, size_t count) {
  size_t need = 0;
  opf_status s = opf_field_size_i(c, inst, field, &need);
  if (s != OPF_OK) return s;
  if (need == 0) return OPF_OK;  // e.g. line fields of a network without lines
  if (!dst) return fail(c, OPF_E_INVALID, "dst is NULL");
  if (count < need) return fail(c, OPF_E_INVALID, "dst too small: need " + std::to_string(need));
  const Inst& x = c->inst[inst];
  if (c->precision == 0)
    launch_export(kargs(x, x.st64, x.geom64), field, dst, c->stream);
  else if (c->bf16_duals)
    launch_export(kargs(x, x.st32b, x.geom32), field, dst, c->stream);
  else
    launch_export(kargs(x, x.st32, x.geom32), field, dst, c->stream);
  HIP_TRY(c, hipGetLastError());
  return OPF_OK;
}

opf_status opf_get_field(opf_ctx* c, int32_t field, double* dst, size_t count) {
  return opf_get_field_i(c, 0, field, dst, count);
}

opf_status opf_set_timing(opf_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
  c->timing = enable != 0;
  for (int i = 0; i < OPF_KERNEL_COUNT; ++i) {
    c->t_ms[i] = 0.0;
    c->t_n[i] = 0;
  }
  return OPF_OK;
}

opf_status opf_kernel_times(opf_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return fail(c, OPF_E_INVALID, "NULL argument");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      c->t_ms[p.kind] += t;
      c->t_n[p.kind] += 1;
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
  for (int i = 0; i < OPF_KERNEL_COUNT; ++i) {
    ms[i] = c->t_ms[i];
    launches[i] = c->t_n[i];
  }
  return OPF_OK;
}

opf_status opf_kernel_bytes(opf_ctx* c, int32_t kernel, double* bytes) {
  if (!c || !bytes) return fail(c, OPF_E_INVALID, "NULL argument");
  if (!c->loaded) return fail(c, OPF_E_STATE, not_loaded_msg(c));
  const double S = c->precision == 0 ? 8.0 : 4.0;
  const double SV = c->precision == 0 ? 8.0 : (c->bf16_duals ? 2.0 : 4.0);
  double total = 0.0;
  for (const Inst& x : c->inst) {
    const double KT = double(x.Kp) * x.T;
    const double L = x.L, N = x.N;
    const double J = double(x.Jnc) * x.T;
    switch (kernel) {
      case OPF_KERNEL_DEVICES:
        // per device and period: read p, theta, averaged dual, both node
        // averages and a parameter; write p, theta, averaged dual
        total += J * 9.0 * S;
        break;
      case OPF_KERNEL_SWEEP:
        // per (k, l, t): read and write P, Tm (S each) and V1, V2 (SV each);
        // per (k, n, t): read and write U, W, thetabar
        total += KT * (L * 2.0 * (2.0 * S + 2.0 * SV) + N * 6.0 * S);
        break;
      case OPF_KERNEL_RESCALE:
        total += KT * N * 4.0 * S;
        break;
      default:
        break;
    }
  }
  *bytes = total;
  return OPF_OK;
}

opf_status opf_autotune(opf_ctx* c, int32_t trials, const char* cache_path, opf_tuning* out) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!c->loaded) return fail(c, OPF_E_STATE, not_loaded_msg(c));
  if (trials < 1) return fail(c, OPF_E_INVALID, "trials must be >= 1");
  // cache key: device, precision, shape of the loaded instances
  hipDeviceProp_t prop;
  int dev = 0;
  HIP_TRY(c, hipGetDevice(&dev));
  HIP_TRY(c, hipGetDeviceProperties(&prop, dev));
  int64_t sN = 0, sL = 0, sKT = 0;
  for (const Inst& x : c->inst) {
    sN += int64_t(x.N) * x.T;
    sL += int64_t(x.L) * x.T;
    sKT += int64_t(x.Kp) * x.T;
  }
  std::ostringstream key;
  key << prop.gcnArchName << "|p" << c->precision << (c->bf16_duals ? "b" : "") << "|n"
      << c->inst.size() << "|NT" << sN << "|LT" << sL << "|KT" << sKT;
  opf_tuning best{};
  best.ms_per_iter = 1e300;
  best.tile_groups = 1;
  bool cached = false;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string k;
    int shift, tiled, groups;
    double gf, ms;
    while (in >> k >> shift >> gf >> tiled >> groups >> ms)
      if (k == key.str()) {
        best.lanes_shift = shift;
        best.grid_factor = gf;
        best.tiled = tiled;
        best.tile_groups = std::max(1, std::min(8, groups));
        best.ms_per_iter = ms;
        cached = true;
      }
  }
  if (!cached) {
    // trials run untimed full iterations whatever the stopping options: no
    // instance may stop (converged or at max_iter) and turn later trials into
    // no-ops; options and the timing switch come back on every exit
    struct Restore {
      opf_ctx* c;
      opf_options opt;
      bool timing;
      ~Restore() {
        c->opt = opt;
        c->timing = timing;
      }
    } restore{c, c->opt, c->timing};
    c->timing = false;
    c->opt.max_iter = INT32_MAX;
    c->opt.min_iter = INT32_MAX;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    bool tiles_possible = true;  // every instance has clusters
    for (const Inst& x : c->inst) tiles_possible = tiles_possible && x.topo.Q > 0;
    // candidates: node rows (lanes per row x grid) and, where the clusters
    // exist, the tiled sweep (grid x period groups per work item)
    struct Cand {
      int tm, shift, groups;
      double gf;
    };
    std::vector<Cand> cands;
    for (int shift = -1; shift <= 1; ++shift)
      for (double gf : {0.5, 1.0, 2.0}) cands.push_back({0, shift, 1, gf});
    if (tiles_possible)
      for (int groups : {1, 2, 4, 8})
        for (double gf : {0.5, 1.0, 2.0}) cands.push_back({1, 0, groups, gf});
    for (const Cand& cd : cands) {
      const int shift = cd.shift;
      const double gf = cd.gf;
      c->tile_mode = cd.tm;
      c->tile_groups = cd.groups;
      c->lanes_shift = shift;
      c->grid_factor = gf;
      opf_status s = refresh_geometry(c);
      if (s != OPF_OK) return s;
      s = reset_state(c);
      if (s != OPF_OK) return s;
      enqueue_n(c, 2, false, c->host_iter);  // warm-up
      c->host_iter += 2;
      HIP_TRY(c, hipEventRecord(e0, c->stream));
      enqueue_n(c, trials, false, c->host_iter);
      c->host_iter += trials;
      HIP_TRY(c, hipEventRecord(e1, c->stream));
      HIP_TRY(c, hipEventSynchronize(e1));
      float ms = 0.0f;
      HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
      const double per = double(ms) / trials;
      if (per < best.ms_per_iter) {
        best.ms_per_iter = per;
        best.lanes_shift = shift;
        best.grid_factor = gf;
        best.tiled = c->tile_mode;
        best.tile_groups = cd.groups;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (cache_path) {
      std::ofstream outf(cache_path, std::ios::app);
      outf << key.str() << " " << best.lanes_shift << " " << best.grid_factor << " "
           << best.tiled << " " << best.tile_groups << " " << best.ms_per_iter << "\n";
    }
  }
  c->lanes_shift = best.lanes_shift;
  c->grid_factor = best.grid_factor;
  c->tile_mode = best.tiled;
  c->tile_groups = best.tile_groups;
  opf_status s = refresh_geometry(c);
  if (s != OPF_OK) return s;
  s = reset_state(c);
  if (s != OPF_OK) return s;
  best.from_cache = cached ? 1 : 0;
  if (out) *out = best;
  return OPF_OK;
}

opf_status opf_state_layout(opf_ctx* c, int32_t instance, opf_layout* out) {
  opf_status s = check_inst(c, instance);
  if (s != OPF_OK) return s;
  if (!out) return fail(c, OPF_E_INVALID, "out is NULL");
  s = read_ctls(c);
  if (s != OPF_OK) return s;
  const Inst& x = c->inst[instance];
  const int cur = c->h_ctl[instance].cur;
  std::memset(out, 0, sizeof(*out));
  out->N = x.N;
  out->T = x.T;
  out->K = x.K;
  out->Kpp = x.Kpp;
  out->L = x.L;
  out->Jnc = x.Jnc;
  out->state_dtype = c->precision == 0 ? OPF_F64 : OPF_F32;
  out->dual_dtype = c->precision == 0 ? OPF_F64 : (c->bf16_duals ? OPF_BF16 : OPF_F32);
  out->chunk = kChunk;
  out->Ldc = x.Ldc;
  out->Zc = x.Zc;
  auto off = [&](const void* p) { return size_t(static_cast<const char*>(p) - c->ws); };
  auto fill = [&](const auto& st) {
    const auto& b = st.buf[cur];
    out->P = off(b.P);
    out->Tm = off(b.Tm);
    out->V1 = off(b.V1);
    out->V2 = off(b.V2);
    out->Td = off(b.Td);
    out->Hd = off(b.Hd);
    out->Tz = off(b.Tz);
    out->U = off(b.U);
    out->W = off(b.W);
    out->TB = off(b.TB);
    out->pnc = off(st.pnc);
    out->thnc = off(st.thnc);
    out->vbar = off(st.vbar);
  };
  if (c->precision == 0)
    fill(x.st64);
  else if (c->bf16_duals)
    fill(x.st32b);
  else
    fill(x.st32);
  return OPF_OK;
}

opf_status opf_state_size(opf_ctx* c, size_t* bytes) {
  opf_status s = state_check(c);
  if (s != OPF_OK) return s;
  if (!bytes) return fail(c, OPF_E_INVALID, "bytes is NULL");
  *bytes = kBlobHead + snap_layout(c->inst[0], c->precision).total;
  return OPF_OK;
}

opf_status opf_get_state(opf_ctx* c, void* dst, size_t bytes) {
  size_t need = 0;
  opf_status s = opf_state_size(c, &need);
  if (s != OPF_OK) return s;
  if (!dst) return fail(c, OPF_E_INVALID, "dst is NULL");
  if (bytes < need) return fail(c, OPF_E_INVALID, "dst too small: need " + std::to_string(need));
  s = read_ctls(c);
  if (s != OPF_OK) return s;
  const Inst& x = c->inst[0];
  const Ctl& h = c->h_ctl[0];
  BlobHead hd{};
  std::memcpy(hd.magic, "OPFSTATE", 8);
  hd.version = 1;
  hd.precision = c->precision;
  hd.N = x.N;
  hd.T = x.T;
  hd.K = x.K;
  hd.L = x.L;
  hd.Jnc = x.Jnc;
  hd.nR = x.nR;
  hd.B = x.B;
  hd.Ldc = x.Ldc;
  hd.n_chg = x.n_chg;
  hd.Zc = x.Zc;
  hd.topo_hash = x.topo_hash;
  hd.rho_p = h.rho_p;
  hd.rho_th = h.rho_th;
  hd.su = h.su;
  hd.sv = h.sv;
  char* blob = static_cast<char*>(dst);
  HIP_TRY(c, hipMemcpyAsync(blob, &hd, sizeof(hd), hipMemcpyDefault, c->stream));
  const SnapLayout sl = snap_layout(x, c->precision);
  s = c->precision == 0 ? state_copy<double>(c, x, h.cur, blob, true, sl)
                        : state_copy<float>(c, x, h.cur, blob, true, sl);
  if (s != OPF_OK) return s;
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return OPF_OK;
}

opf_status opf_set_state(opf_ctx* c, const void* src, size_t bytes) {
  opf_status s = state_check(c);
  if (s != OPF_OK) return s;
  if (!src) return fail(c, OPF_E_INVALID, "src is NULL");
  if (bytes < kBlobHead) return fail(c, OPF_E_INVALID, "state too small");
  BlobHead hd{};
  HIP_TRY(c, hipMemcpy(&hd, src, sizeof(hd), hipMemcpyDefault));
  const Inst& x = c->inst[0];
  if (std::memcmp(hd.magic, "OPFSTATE", 8) != 0 || hd.version != 1)
    return fail(c, OPF_E_INVALID, "not a state exported by opf_get_state");
  if (hd.N != x.N || hd.T != x.T || hd.K != x.K || hd.L != x.L || hd.Jnc != x.Jnc ||
      hd.nR != x.nR || hd.B != x.B || hd.Ldc != x.Ldc ||
      hd.n_chg != x.n_chg || hd.Zc != x.Zc)
    return fail(c, OPF_E_INVALID, "state was exported from a network of another shape");
  if (hd.topo_hash != x.topo_hash)
    return fail(c, OPF_E_INVALID,
                "state was exported from a network of another structure (lines, outages or "
                "device nodes differ)");
  if (!(hd.precision == 0 ? c->has64 : c->has32))
    return fail(c, OPF_E_INVALID, "state precision is not held by this context");
  if (!(hd.rho_p > 0.0 && hd.rho_th > 0.0 && std::isfinite(hd.rho_p) && std::isfinite(hd.rho_th) &&
        hd.su > 0.0 && hd.sv > 0.0 && std::isfinite(hd.su) && std::isfinite(hd.sv)))
    return fail(c, OPF_E_INVALID, "state penalties are not positive");
  const SnapLayout sl = snap_layout(x, hd.precision);
  if (bytes < kBlobHead + sl.total)
    return fail(c, OPF_E_INVALID, "state too small: need " + std::to_string(kBlobHead + sl.total));
  s = reset_state(c);
  if (s != OPF_OK) return s;
  char* blob = const_cast<char*>(static_cast<const char*>(src));
  s = hd.precision == 0 ? state_copy<double>(c, x, 0, blob, false, sl)
                        : state_copy<float>(c, x, 0, blob, false, sl);
  if (s != OPF_OK) return s;
  Ctl& h = c->h_ctl[0];
  h.rho_p = hd.rho_p;
  h.rho_th = hd.rho_th;
  h.su = hd.su;
  h.sv = hd.sv;
  h.precision = hd.precision;
  HIP_TRY(c, hipMemcpyAsync(x.ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->precision = hd.precision;
  return OPF_OK;
}

opf_status opf_tape_workspace_size(opf_ctx* c, int32_t n_iters, int32_t checkpoint_every,
                                   size_t* bytes) {
  opf_status s = tape_check(c);
  if (s != OPF_OK) return s;
  if (!bytes) return fail(c, OPF_E_INVALID, "bytes is NULL");
  if (n_iters < 1 || checkpoint_every < 1)
    return fail(c, OPF_E_INVALID, "need n_iters >= 1 and checkpoint_every >= 1");
  *bytes = plan_tape(c->inst[0], c->has32 ? 1 : 0, n_iters, checkpoint_every).total;
  return OPF_OK;
}

opf_status opf_tape_forward(opf_ctx* c, int32_t n_iters, int32_t checkpoint_every,
                            void* d_tape, size_t bytes) {
  size_t need = 0;
  opf_status s = opf_tape_workspace_size(c, n_iters, checkpoint_every, &need);
  if (s != OPF_OK) return s;
  if (!d_tape) return fail(c, OPF_E_INVALID, "tape workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_tape) % kAlign != 0)
    return fail(c, OPF_E_INVALID, "tape workspace must be 256-byte aligned");
  if (bytes < need)
    return fail(c, OPF_E_INVALID, "tape workspace too small: need " + std::to_string(need));
  // the run starts from the zero iterate in the configured state precision
  c->tape = plan_tape(c->inst[0], c->has32 ? 1 : 0, n_iters, checkpoint_every);
  c->tape.base = static_cast<char*>(d_tape);
  c->tape.bytes = bytes;
  return c->tape.precision == 0 ? tape_forward<double>(c, n_iters, checkpoint_every, false, 0, nullptr)
                                : tape_forward<float>(c, n_iters, checkpoint_every, false, 0, nullptr);
}

opf_status opf_tape_forward_warm(opf_ctx* c, int32_t min_iters, int32_t max_iters,
                                 int32_t checkpoint_every, void* d_tape, size_t bytes,
                                 int32_t* n_run) {
  size_t need = 0;
  opf_status s = opf_tape_workspace_size(c, max_iters, checkpoint_every, &need);
  if (s != OPF_OK) return s;
  if (min_iters < 0 || min_iters > max_iters)
    return fail(c, OPF_E_INVALID, "need 0 <= min_iters <= max_iters");
  if (!d_tape) return fail(c, OPF_E_INVALID, "tape workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_tape) % kAlign != 0)
    return fail(c, OPF_E_INVALID, "tape workspace must be 256-byte aligned");
  if (bytes < need)
    return fail(c, OPF_E_INVALID, "tape workspace too small: need " + std::to_string(need));
  s = read_ctls(c);
  if (s != OPF_OK) return s;
  const int active = c->h_ctl[0].precision;
  if ((active == 0 ? 0 : 1) != (c->has32 ? 1 : 0))
    return fail(c, OPF_E_STATE, "the current iterate is not in the configured state precision");
  c->tape = plan_tape(c->inst[0], c->has32 ? 1 : 0, max_iters, checkpoint_every);
  c->tape.base = static_cast<char*>(d_tape);
  c->tape.bytes = bytes;
  return c->tape.precision == 0
             ? tape_forward<double>(c, max_iters, checkpoint_every, true, min_iters, n_run)
             : tape_forward<float>(c, max_iters, checkpoint_every, true, min_iters, n_run);
}

opf_status opf_adjoint(opf_ctx* c, const double* d_cot_power, double cot_objective,
                       double* d_grad_load, double* d_grad_cap, double* d_grad_pmax) {
  opf_status s = tape_check(c);
  if (s != OPF_OK) return s;
  if (!c->tape.ready) return fail(c, OPF_E_STATE, "no tape: call opf_tape_forward first");
  if (!std::isfinite(cot_objective)) return fail(c, OPF_E_INVALID, "cot_objective not finite");
  return c->tape.precision == 0
             ? adjoint<double>(c, d_cot_power, cot_objective, d_grad_load, d_grad_cap, d_grad_pmax)
             : adjoint<float>(c, d_cot_power, cot_objective, d_grad_load, d_grad_cap, d_grad_pmax);
}

const char* opf_last_error(opf_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

void opf_destroy(opf_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  release_static(c);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);
  if (c->h_rec) (void)hipHostFree(c->h_rec);
  if (c->h_int) (void)hipHostFree(c->h_int);
  delete c;
}

}  // extern "C"
