// Host side of the C ABI declared in include/opf.h: validation, the
// CSR-by-node structure, workspace layout, launch sequencing of one
// message-passing iteration (Section 3.2 of arXiv 2410.17203), HIP-graph
// blocks of iterations, the solve loop with FP64 polishing, and per-kernel
// event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/opf.h"
#include "opf_internal.h"

using namespace opf;

namespace {

constexpr size_t kAlign = 256;
// Upper bound of the sweep grid (partials are sized for it); the grid used
// is the number of blocks resident at once on the device.
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

// Offsets of one precision's iterate inside the workspace.
struct BufOffsets {
  size_t P, Tm, V1, V2, Td, U, W, TB;
};
struct StateOffsets {
  BufOffsets buf[2];
  size_t avgW, avgTB, pnc, thnc, vbar, ramp, bat;
};

struct Timed {
  int kind;
  hipEvent_t a, b;
};

}  // namespace

struct opf_ctx {
  opf_options opt{};
  std::string err;
  hipStream_t stream = nullptr;
  bool loaded = false;
  // sizes
  int N = 0, T = 0, K = 0, Kp = 0, Kpp = 0, L = 0, G = 0, D = 0, B = 0, Jnc = 0, nR = 0;
  double eps_eff = 0.0, rms_norm = 1.0;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Topo topo{};
  Geom geom64{}, geom32{};
  bool has64 = false, has32 = false;
  State<double, double> st64{};
  State<float, float> st32{};
  State<float, bf16_t> st32b{};
  int precision = 0;  // 0 = FP64 iterate active, 1 = FP32
  bool bf16_duals = false;
  int64_t host_iter = 0;
  Ctl* ctl = nullptr;
  Rec* ring = nullptr;
  // pinned readback buffers
  Ctl* h_ctl = nullptr;
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

// Validates the network; on success fills the derived sizes into c (not
// committed until load succeeds).
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
    if (!(n->line_sus[l] > 0.0) || !finite(n->line_sus[l]))
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
  for (int g = 0; g < n->G; ++g) {
    if (!node_ok(n->gen_node[g])) return fail(c, OPF_E_INVALID, "generator node out of range");
    deg[n->gen_node[g]]++;
    if (!(n->gen_c2[g] > 0.0) || !finite(n->gen_c2[g]) || !finite(n->gen_c1[g]))
      return fail(c, OPF_E_INVALID, "generator costs must be finite with c2 > 0");
    const double r = n->gen_ramp[g];
    if (std::isnan(r)) return fail(c, OPF_E_INVALID, "generator ramp is NaN");
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

void make_geom(opf_ctx* c, int vec, Geom& g) {
  g.nv = c->Kpp / vec;
  g.n_nc_blocks = (c->Jnc + 3) / 4;
  int lpr = 1;
  while (lpr < g.nv && lpr < kWave) lpr *= 2;
  g.lanes_per_row = lpr;
  g.rows_per_grp = (kBlock / kWave) * (kWave / lpr);
  const int64_t NT = int64_t(c->N) * c->T;
  g.n_grps = (NT + g.rows_per_grp - 1) / g.rows_per_grp;
  g.n_sweep_blocks = std::max(8, round8(std::min<int64_t>(g.n_grps, kMaxSweepBlocks)));
  g.inner_iters = c->opt.inner_iters;
  g.omega_scale = c->opt.inner_omega_scale;
}

template <typename R, typename VT>
void state_offsets(opf_ctx* c, Layout& lay, StateOffsets& o) {
  const size_t line = size_t(c->L) * c->T * c->Kpp;
  const size_t node = size_t(c->N) * c->T * c->Kpp;
  for (int i = 0; i < 2; ++i) {
    BufOffsets& b = o.buf[i];
    b.P = lay.take(line * sizeof(R));
    b.Tm = lay.take(line * sizeof(R));
    b.V1 = lay.take(line * sizeof(VT));
    b.V2 = lay.take(line * sizeof(VT));
    b.Td = lay.take(size_t(c->T) * c->Kpp * sizeof(R));
    b.U = lay.take(node * sizeof(R));
    b.W = lay.take(node * sizeof(R));
    b.TB = lay.take(node * sizeof(R));
  }
  o.avgW = lay.take(size_t(c->N) * c->T * sizeof(R));
  o.avgTB = lay.take(size_t(c->N) * c->T * sizeof(R));
  const size_t nc = size_t(c->Jnc) * c->T;
  o.pnc = lay.take(nc * sizeof(R));
  o.thnc = lay.take(nc * sizeof(R));
  o.vbar = lay.take(nc * sizeof(R));
  o.ramp = lay.take(4 * size_t(c->nR) * c->T * sizeof(R));
  o.bat = lay.take(6 * size_t(c->B) * c->T * sizeof(R));
}

template <typename R, typename VT>
State<R, VT> state_ptrs(char* ws, const StateOffsets& o) {
  State<R, VT> s;
  for (int i = 0; i < 2; ++i) {
    const BufOffsets& b = o.buf[i];
    Buf<R, VT>& d = s.buf[i];
    d.P = reinterpret_cast<R*>(ws + b.P);
    d.Tm = reinterpret_cast<R*>(ws + b.Tm);
    d.V1 = reinterpret_cast<VT*>(ws + b.V1);
    d.V2 = reinterpret_cast<VT*>(ws + b.V2);
    d.Td = reinterpret_cast<R*>(ws + b.Td);
    d.U = reinterpret_cast<R*>(ws + b.U);
    d.W = reinterpret_cast<R*>(ws + b.W);
    d.TB = reinterpret_cast<R*>(ws + b.TB);
  }
  s.avgW = reinterpret_cast<R*>(ws + o.avgW);
  s.avgTB = reinterpret_cast<R*>(ws + o.avgTB);
  s.pnc = reinterpret_cast<R*>(ws + o.pnc);
  s.thnc = reinterpret_cast<R*>(ws + o.thnc);
  s.vbar = reinterpret_cast<R*>(ws + o.vbar);
  s.ramp_st = reinterpret_cast<R*>(ws + o.ramp);
  s.bat_st = reinterpret_cast<R*>(ws + o.bat);
  return s;
}

// Everything the workspace holds, in order.
struct Plan {
  Layout lay;
  size_t ctl, ring;
  size_t line_from, line_to, sus, cap, outage_k, node_lptr, node_lterm, node_nptr, node_nterm, deg,
      nc_node, ramp_idx, gen_c2, gen_c1, gen_pmin, gen_pmax, gen_ramp, load_d, bat_P, bat_dur,
      bat_eta, bat_alpha;
  size_t part_sweep, part_nc;
  size_t state_begin, state_end;
  bool has64 = false, has32 = false;
  StateOffsets o64{}, o32{};
};

void make_plan(opf_ctx* c, Plan& p) {
  Layout& L = p.lay;
  p.ctl = L.take(sizeof(Ctl));
  p.ring = L.take(sizeof(Rec) * kRing);
  const size_t Li = size_t(c->L), Ni = size_t(c->N), Gi = size_t(c->G), T = size_t(c->T);
  p.line_from = L.take(Li * 4);
  p.line_to = L.take(Li * 4);
  p.sus = L.take(Li * 8);
  p.cap = L.take(Li * 8);
  p.outage_k = L.take(size_t(c->Kpp) * 4);
  p.node_lptr = L.take((Ni + 1) * 4);
  p.node_lterm = L.take(4 * Li * 4);
  p.node_nptr = L.take((Ni + 1) * 4);
  p.node_nterm = L.take(size_t(c->Jnc) * 4);
  p.deg = L.take(Ni * 8);
  p.nc_node = L.take(size_t(c->Jnc) * 4);
  p.ramp_idx = L.take(Gi * 4);
  p.gen_c2 = L.take(Gi * 8);
  p.gen_c1 = L.take(Gi * 8);
  p.gen_pmin = L.take(Gi * T * 8);
  p.gen_pmax = L.take(Gi * T * 8);
  p.gen_ramp = L.take(Gi * 8);
  p.load_d = L.take(size_t(c->D) * T * 8);
  p.bat_P = L.take(size_t(c->B) * 8);
  p.bat_dur = L.take(size_t(c->B) * 8);
  p.bat_eta = L.take(size_t(c->B) * 8);
  p.bat_alpha = L.take(size_t(c->B) * 8);
  Geom g64{}, g32{};
  make_geom(c, 2, g64);
  make_geom(c, 4, g32);
  const int nsb = std::max(g64.n_sweep_blocks, g32.n_sweep_blocks);
  p.part_sweep = L.take(size_t(nsb) * 5 * 8);
  p.part_nc = L.take(size_t(std::max(g64.n_nc_blocks, 1)) * 2 * 8);
  p.state_begin = L.total;
  p.has32 = c->opt.state_dtype == OPF_F32;
  p.has64 = !p.has32 || c->opt.polish_fp64;
  if (p.has64) state_offsets<double, double>(c, L, p.o64);
  if (p.has32) {
    if (c->opt.dual_dtype == OPF_BF16)
      state_offsets<float, bf16_t>(c, L, p.o32);
    else
      state_offsets<float, float>(c, L, p.o32);
  }
  p.state_end = L.total;
}

void set_sizes(opf_ctx* c, const opf_network* n) {
  c->N = n->N;
  c->T = n->T;
  c->K = n->K;
  c->Kp = n->K + 1;
  c->Kpp = (c->Kp + 3) / 4 * 4;
  c->L = n->L;
  c->G = n->G;
  c->D = n->D;
  c->B = n->B;
  c->Jnc = n->G + n->D + n->B;
  c->nR = 0;
  if (n->T > 1)
    for (int g = 0; g < n->G; ++g)
      if (n->gen_ramp[g] > 0.0 && std::isfinite(n->gen_ramp[g])) c->nR++;
}

template <typename R, typename VT>
KArgs<R, VT> kargs(opf_ctx* c, const State<R, VT>& st, const Geom& g) {
  KArgs<R, VT> a;
  a.tp = c->topo;
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

template <typename R, typename VT>
void enqueue_iter(opf_ctx* c, const KArgs<R, VT>& a, int64_t iter_index, bool capturing) {
  // iter_index: 0-based index of this iteration since the start
  timed(c, OPF_KERNEL_DEVICES, [&] { launch_devices(a, c->stream); }, capturing);
  timed(c, OPF_KERNEL_SWEEP, [&] { launch_sweep(a, c->stream); }, capturing);
  timed(c, OPF_KERNEL_FINALIZE, [&] { launch_finalize(a, c->stream); }, capturing);
  const int ae = c->opt.adapt_every;
  if (ae > 0 && (iter_index + 1) % ae == 0)
    timed(c, OPF_KERNEL_RESCALE, [&] { launch_rescale(a, c->stream); }, capturing);
}

void enqueue_n(opf_ctx* c, int n, bool capturing, int64_t start) {
  for (int i = 0; i < n; ++i) {
    const int64_t it = start + i;
    if (c->precision == 0)
      enqueue_iter(c, kargs(c, c->st64, c->geom64), it, capturing);
    else if (c->bf16_duals)
      enqueue_iter(c, kargs(c, c->st32b, c->geom32), it, capturing);
    else
      enqueue_iter(c, kargs(c, c->st32, c->geom32), it, capturing);
  }
}

opf_status read_ctl(opf_ctx* c) {
  HIP_TRY(c, hipMemcpyAsync(c->h_ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return OPF_OK;
}

opf_status last_record(opf_ctx* c, opf_resid* out) {
  opf_status s = read_ctl(c);
  if (s != OPF_OK) return s;
  std::memset(out, 0, sizeof(*out));
  const int iter = c->h_ctl->iter;
  const int ce = std::max(1, c->opt.check_every);
  const int last = iter - iter % ce;
  out->iter = iter;
  out->rho_p = c->h_ctl->rho_p;
  out->rho_theta = c->h_ctl->rho_th;
  out->threshold = c->eps_eff;
  out->precision = c->precision == 0 ? OPF_F64 : OPF_F32;
  if (last <= 0) return OPF_OK;
  HIP_TRY(c, hipMemcpyAsync(c->h_rec, c->ring + (last - 1) % kRing, sizeof(Rec),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const Rec& r = *c->h_rec;
  out->primal_p = r.primal_p;
  out->primal_theta = r.primal_th;
  out->dual_p = r.dual_p;
  out->dual_theta = r.dual_th;
  out->rms_primal = r.rms_primal;
  out->rms_dual = r.rms_dual;
  out->threshold = r.threshold;
  out->objective = r.objective;
  out->rho_p = r.rho_p;
  out->rho_theta = r.rho_th;
  out->converged = r.converged;
  out->precision = r.precision == 0 ? OPF_F64 : OPF_F32;
  return OPF_OK;
}

opf_status widen_to_fp64(opf_ctx* c) {
  KArgs<double, double> dst = kargs(c, c->st64, c->geom64);
  if (c->bf16_duals)
    launch_widen(kargs(c, c->st32b, c->geom32), dst, c->stream);
  else
    launch_widen(kargs(c, c->st32, c->geom32), dst, c->stream);
  HIP_TRY(c, hipGetLastError());
  *c->h_int = 0;
  HIP_TRY(c, hipMemcpyAsync(&c->ctl->precision, c->h_int, sizeof(int32_t), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->precision = 0;
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
  if (o.inner_iters < 1 || !(o.inner_omega_scale > 0))
    return fail(nullptr, OPF_E_INVALID, "need inner_iters >= 1 and inner_omega_scale > 0");
  opf_ctx* c = new opf_ctx();
  c->opt = o;
  c->stream = reinterpret_cast<hipStream_t>(o.hip_stream);
  c->bf16_duals = o.dual_dtype == OPF_BF16;
  *out = c;
  return OPF_OK;
}

opf_status opf_workspace_size(opf_ctx* c, const opf_network* n, size_t* bytes) {
  if (!c || !bytes) return fail(c, OPF_E_INVALID, "NULL argument");
  opf_ctx probe;
  probe.opt = c->opt;
  opf_status s = validate(&probe, n);
  if (s != OPF_OK) return fail(c, s, probe.err);
  set_sizes(&probe, n);
  Plan p;
  make_plan(&probe, p);
  *bytes = p.lay.total;
  return OPF_OK;
}

opf_status opf_load_network(opf_ctx* c, const opf_network* n, void* d_ws, size_t bytes) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!d_ws) return fail(c, OPF_E_INVALID, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign)
    return fail(c, OPF_E_INVALID, "workspace must be 256-byte aligned");
  opf_ctx probe;
  probe.opt = c->opt;
  opf_status s = validate(&probe, n);
  if (s != OPF_OK) return fail(c, s, probe.err);
  set_sizes(&probe, n);
  Plan p;
  make_plan(&probe, p);
  if (bytes < p.lay.total)
    return fail(c, OPF_E_OOM, "workspace too small: need " + std::to_string(p.lay.total) + " bytes");

  // ---- host-side derived data --------------------------------------------
  const int N = probe.N, T = probe.T, L = probe.L, G = probe.G, D = probe.D, B = probe.B;
  const int Jnc = probe.Jnc, Kpp = probe.Kpp;
  std::vector<int32_t> outage_k(Kpp, -1);
  for (int k = 1; k <= probe.K; ++k) outage_k[k] = n->outage[k - 1];
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
  std::vector<int32_t> ramp_idx(G, -1);
  {
    int r = 0;
    if (T > 1)
      for (int g = 0; g < G; ++g)
        if (n->gen_ramp[g] > 0.0 && std::isfinite(n->gen_ramp[g])) ramp_idx[g] = r++;
  }
  double lsum = 0.0;
  for (size_t i = 0; i < size_t(D) * T; ++i) lsum += n->load_d[i] * n->load_d[i];
  const double load_rms = (size_t(D) * T > 0) ? std::sqrt(lsum / double(size_t(D) * T)) : 1.0;

  // pinned readback buffers (first load only)
  if (!c->h_ctl) {
    HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_ctl), sizeof(Ctl)));
    HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_rec), sizeof(Rec) * kRing));
    HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&c->h_int), 64));
  }

  // ---- commit ---------------------------------------------------------------
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->N = probe.N; c->T = T; c->K = probe.K; c->Kp = probe.Kp; c->Kpp = Kpp;
  c->L = L; c->G = G; c->D = D; c->B = B; c->Jnc = Jnc; c->nR = probe.nR;
  c->ws = static_cast<char*>(d_ws);
  c->ws_bytes = bytes;
  char* ws = c->ws;
  auto up = [&](size_t off, const void* src, size_t nbytes) -> hipError_t {
    if (nbytes == 0) return hipSuccess;
    return hipMemcpyAsync(ws + off, src, nbytes, hipMemcpyHostToDevice, c->stream);
  };
  HIP_TRY(c, hipMemsetAsync(ws, 0, p.lay.total, c->stream));
  HIP_TRY(c, up(p.line_from, n->line_from, size_t(L) * 4));
  HIP_TRY(c, up(p.line_to, n->line_to, size_t(L) * 4));
  HIP_TRY(c, up(p.sus, n->line_sus, size_t(L) * 8));
  HIP_TRY(c, up(p.cap, n->line_cap, size_t(L) * 8));
  HIP_TRY(c, up(p.outage_k, outage_k.data(), size_t(Kpp) * 4));
  HIP_TRY(c, up(p.node_lptr, lptr.data(), size_t(N + 1) * 4));
  HIP_TRY(c, up(p.node_lterm, lterm.data(), lterm.size() * 4));
  HIP_TRY(c, up(p.node_nptr, nptr.data(), size_t(N + 1) * 4));
  HIP_TRY(c, up(p.node_nterm, nterm.data(), nterm.size() * 4));
  HIP_TRY(c, up(p.deg, deg.data(), size_t(N) * 8));
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

  Topo& tp = c->topo;
  tp.N = N; tp.T = T; tp.K = probe.K; tp.Kp = probe.Kp; tp.Kpp = Kpp; tp.L = L; tp.G = G;
  tp.D = D; tp.B = B; tp.Jnc = Jnc; tp.nR = probe.nR;
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

  c->ctl = reinterpret_cast<Ctl*>(ws + p.ctl);
  c->ring = reinterpret_cast<Rec*>(ws + p.ring);
  auto fill_geom = [&](Geom& g, int vec, int resident) {
    make_geom(c, vec, g);
    if (resident >= 8) {
      const int cap = std::min(kMaxSweepBlocks, resident / 8 * 8);
      g.n_sweep_blocks = std::max(8, std::min(g.n_sweep_blocks, cap));
    }
    g.part_sweep = reinterpret_cast<double*>(ws + p.part_sweep);
    g.part_nc = reinterpret_cast<double*>(ws + p.part_nc);
    g.ctl = c->ctl;
    g.ring = c->ring;
  };
  fill_geom(c->geom64, 2, sweep_resident_blocks<double, double>());
  fill_geom(c->geom32, 4, c->bf16_duals ? sweep_resident_blocks<float, bf16_t>()
                                       : sweep_resident_blocks<float, float>());
  c->has64 = p.has64;
  c->has32 = p.has32;
  if (p.has64) c->st64 = state_ptrs<double, double>(ws, p.o64);
  if (p.has32) {
    if (c->bf16_duals)
      c->st32b = state_ptrs<float, bf16_t>(ws, p.o32);
    else
      c->st32 = state_ptrs<float, float>(ws, p.o32);
  }
  c->precision = p.has32 ? 1 : 0;
  c->eps_eff = c->opt.eps * (c->opt.eps_relative ? load_rms : 1.0);
  const double J = 2.0 * L + Jnc;
  c->rms_norm = std::sqrt(2.0 * J * T * double(probe.Kp));
  Ctl& h = *c->h_ctl;
  std::memset(&h, 0, sizeof(Ctl));
  h.rho_p = c->opt.rho_p;
  h.rho_th = c->opt.rho_theta;
  h.su = 1.0;
  h.sv = 1.0;
  h.eps_eff = c->eps_eff;
  h.rms_norm = c->rms_norm;
  h.mu = c->opt.mu;
  h.gamma = c->opt.gamma;
  h.adapt_every = c->opt.adapt_every;
  h.check_every = c->opt.check_every;
  h.max_iter = c->opt.max_iter;
  h.min_iter = c->opt.min_iter;
  h.precision = c->precision;
  HIP_TRY(c, hipMemcpyAsync(c->ctl, &h, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->host_iter = 0;
  c->loaded = true;
  return OPF_OK;
}

opf_status opf_iterate(opf_ctx* c, int32_t n) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!c->loaded) return fail(c, OPF_E_STATE, "no network loaded");
  if (n < 0) return fail(c, OPF_E_INVALID, "n_iters must be >= 0");
  enqueue_n(c, n, false, c->host_iter);
  c->host_iter += n;
  HIP_TRY(c, hipGetLastError());
  return OPF_OK;
}

opf_status opf_solve(opf_ctx* c, opf_resid* out) {
  if (!c) return fail(nullptr, OPF_E_INVALID, "ctx is NULL");
  if (!c->loaded) return fail(c, OPF_E_STATE, "no network loaded");
  const int blk = c->opt.block_iters;
  const int ae = c->opt.adapt_every;
  // graphs need a capturable (non-null) stream and blocks aligned to the
  // penalty-update period
  const bool graph_ok = c->opt.use_graphs && !c->timing && c->stream != nullptr &&
                        (ae == 0 || blk % ae == 0);
  opf_status s = read_ctl(c);
  if (s != OPF_OK) return s;
  while (!c->h_ctl->done && c->h_ctl->iter < c->opt.max_iter) {
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
    s = read_ctl(c);
    if (s != OPF_OK) return s;
    if (c->h_ctl->numeric_bad) break;
    if (c->precision == 1 && c->opt.polish_fp64 && c->has64 && !c->h_ctl->done) {
      opf_resid r;
      s = last_record(c, &r);
      if (s != OPF_OK) return s;
      if (r.iter > 0 && std::max(r.rms_primal, r.rms_dual) <= c->opt.polish_factor * c->eps_eff) {
        s = widen_to_fp64(c);
        if (s != OPF_OK) return s;
      }
    }
  }
  opf_resid r;
  s = last_record(c, &r);
  if (s != OPF_OK) return s;
  if (out) *out = r;
  if (c->h_ctl->numeric_bad) return fail(c, OPF_E_NUMERIC, "residual became NaN or infinite");
  return c->h_ctl->converged ? OPF_OK : OPF_NOT_CONVERGED;
}

opf_status opf_residuals(opf_ctx* c, opf_resid* out) {
  if (!c || !out) return fail(c, OPF_E_INVALID, "NULL argument");
  if (!c->loaded) return fail(c, OPF_E_STATE, "no network loaded");
  opf_status s = last_record(c, out);
  if (s != OPF_OK) return s;
  if (c->h_ctl->numeric_bad) return fail(c, OPF_E_NUMERIC, "residual became NaN or infinite");
  return OPF_OK;
}

opf_status opf_residual_history(opf_ctx* c, opf_resid* out, int32_t max, int32_t* n) {
  if (!c || !out || !n || max < 0) return fail(c, OPF_E_INVALID, "bad argument");
  if (!c->loaded) return fail(c, OPF_E_STATE, "no network loaded");
  opf_status s = read_ctl(c);
  if (s != OPF_OK) return s;
  const int iter = c->h_ctl->iter;
  const int ce = std::max(1, c->opt.check_every);
  HIP_TRY(c, hipMemcpyAsync(c->h_rec, c->ring, sizeof(Rec) * kRing, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int first = std::max(1, iter - kRing + 1);
  int cnt = 0;
  for (int i = first; i <= iter && cnt < max; ++i) {
    if (i % ce) continue;
    const Rec& r = c->h_rec[(i - 1) % kRing];
    opf_resid& o = out[cnt++];
    std::memset(&o, 0, sizeof(o));
    o.iter = r.iter;
    o.primal_p = r.primal_p;
    o.primal_theta = r.primal_th;
    o.dual_p = r.dual_p;
    o.dual_theta = r.dual_th;
    o.rms_primal = r.rms_primal;
    o.rms_dual = r.rms_dual;
    o.threshold = r.threshold;
    o.objective = r.objective;
    o.rho_p = r.rho_p;
    o.rho_theta = r.rho_th;
    o.converged = r.converged;
    o.precision = r.precision == 0 ? OPF_F64 : OPF_F32;
  }
  *n = cnt;
  return OPF_OK;
}

opf_status opf_field_size(opf_ctx* c, int32_t field, size_t* count) {
  if (!c || !count) return fail(c, OPF_E_INVALID, "NULL argument");
  if (!c->loaded) return fail(c, OPF_E_STATE, "no network loaded");
  const size_t KT = size_t(c->Kp) * c->T;
  if (field >= OPF_FIELD_P && field <= OPF_FIELD_V2)
    *count = KT * c->L;
  else if (field >= OPF_FIELD_U && field <= OPF_FIELD_THBAR)
    *count = KT * c->N;
  else if (field >= OPF_FIELD_PNC && field <= OPF_FIELD_VNC)
    *count = size_t(c->Jnc) * c->T;
  else
    return fail(c, OPF_E_INVALID, "unknown field");
  return OPF_OK;
}

opf_status opf_get_field(opf_ctx* c, int32_t field, double* dst, size_t count) {
  size_t need = 0;
  opf_status s = opf_field_size(c, field, &need);
  if (s != OPF_OK) return s;
  if (!dst) return fail(c, OPF_E_INVALID, "dst is NULL");
  if (count < need) return fail(c, OPF_E_INVALID, "dst too small: need " + std::to_string(need));
  if (c->precision == 0)
    launch_export(kargs(c, c->st64, c->geom64), field, dst, c->stream);
  else if (c->bf16_duals)
    launch_export(kargs(c, c->st32b, c->geom32), field, dst, c->stream);
  else
    launch_export(kargs(c, c->st32, c->geom32), field, dst, c->stream);
  HIP_TRY(c, hipGetLastError());
  return OPF_OK;
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
  if (!c->loaded) return fail(c, OPF_E_STATE, "no network loaded");
  const double S = c->precision == 0 ? 8.0 : 4.0;
  const double SV = c->precision == 0 ? 8.0 : (c->bf16_duals ? 2.0 : 4.0);
  const double KT = double(c->Kp) * c->T;
  const double L = c->L, N = c->N;
  const double J = double(c->Jnc) * c->T;
  switch (kernel) {
    case OPF_KERNEL_DEVICES:
      // per device and period: read p, theta, averaged dual, both node
      // averages and a parameter; write p, theta, averaged dual
      *bytes = J * 9.0 * S;
      break;
    case OPF_KERNEL_SWEEP:
      // per (k, l, t): read and write P, Tm (S each) and V1, V2 (SV each);
      // per (k, n, t): read and write U, W, thetabar
      *bytes = KT * (L * 2.0 * (2.0 * S + 2.0 * SV) + N * 6.0 * S);
      break;
    case OPF_KERNEL_RESCALE:
      *bytes = KT * N * 4.0 * S;
      break;
    default:
      *bytes = 0.0;
  }
  return OPF_OK;
}

const char* opf_last_error(opf_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

void opf_destroy(opf_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
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
