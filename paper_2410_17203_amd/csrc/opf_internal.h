// Internal device-side data structures of the message-passing library.
//
// Data layout in HBM (one instance):
//   line arrays   [T][chunk][L][w]  flow P, mean phase Tm, phase duals V1, V2
//   node arrays   [T][chunk][N][w]  price U, W = pbar + U, thetabar TB
//   node averages [N][T]            mean over contingencies of W and TB
//   device arrays [Jnc][T]          generator/load/battery power, phase and
//                                   the contingency-averaged phase dual
// The K+1 contingencies (padded to Kpp, a multiple of 4) are split into
// chunks of 32 (the last one w = Kpp - 32 c wide).  Within a chunk the w
// contingencies of one line or node are contiguous (128 bytes in FP32, one
// L2 line, so an isolated gather wastes nothing) and
// consecutive lines or nodes follow each other, so a tile of neighbouring
// nodes (or the lines they own) in one period and chunk is one contiguous
// run of memory, and every 16-byte vector of contingencies lies in one chunk.
// Time is outermost.  FP32 and FP64 iterates use the same element indices.
// A line's two phases are stored as their mean Tm; the half difference is
// P / (2 b) for a live line and, for the one outaged line of contingency k,
// a separate [T][Kpp] array Td.  A DC link has no phase relation, so its
// half difference is state of its own: Hd [T][chunk][Ldc][w] over the DC
// links in line order; so is that of a line taken out by a general
// per-contingency change: Tz [T][Zc].  Line and node arrays are double-buffered
// (the sweep reads one buffer and writes the other).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace opf {

constexpr int kBlock = 256;      // threads per block of every kernel
constexpr int kWave = 64;        // CDNA wavefront
constexpr int kRing = 4096;      // residual records kept on the device
constexpr int kMaxAdjInner = 32; // inner iterations the adjoint's clip recorder holds
#ifndef OPF_CHUNK
#define OPF_CHUNK 32
#endif
constexpr int kChunk = OPF_CHUNK; // contingencies per chunk of the line and node arrays
#ifndef OPF_TILE_NODES
#define OPF_TILE_NODES 64
#endif
#ifndef OPF_TILE_LINES
#define OPF_TILE_LINES 128
#endif
constexpr int kTileNodes = OPF_TILE_NODES;  // most nodes in one cluster of the tiled sweep
constexpr int kTileLines = OPF_TILE_LINES;  // most lines touching one cluster
constexpr int kTileDev = 128;               // most generators, loads, batteries in one cluster
#ifndef OPF_TILE_BLOCK
#define OPF_TILE_BLOCK 512
#endif
constexpr int kTileBlock = OPF_TILE_BLOCK;  // threads per workgroup of the tiled sweep
#ifndef OPF_PASS_BYTES
#define OPF_PASS_BYTES 128
#endif
// Contingencies per pass of the tiled sweep: 128 bytes of each row (a chunk
// in FP32, half a chunk in FP64).
template <typename R>
__host__ __device__ constexpr int tile_pass_elems() {
  return OPF_PASS_BYTES / int(sizeof(R)) < kChunk ? OPF_PASS_BYTES / int(sizeof(R)) : kChunk;
}
// Periods that share one pass of the tiled sweep for an instance of Kpp
// (padded) contingencies: where a pass holds all of a period's
// contingencies, as many periods as fill it, at most 4 in FP32 (the LDS
// holds the device values of 4 periods) and 1 in FP64.
template <typename R>
__host__ __device__ inline int tile_group_periods(int Kpp) {
  constexpr int VEC = 16 / int(sizeof(R));
  constexpr int SUB = tile_pass_elems<R>();
  constexpr int NPP = sizeof(R) == 4 ? 4 : 1;
  if (Kpp > SUB) return 1;
  const int nv = (SUB / VEC) / (Kpp / VEC);
  return nv < NPP ? nv : NPP;
}

// Element index of contingency k of item i (a line, count = L, or a node,
// count = N) in period t.
__host__ __device__ inline size_t ck_off(int t, int i, int k, int count, int Kpp) {
  const int c0 = k & ~(kChunk - 1);
  const int w = Kpp - c0 < kChunk ? Kpp - c0 : kChunk;
  return (size_t(t) * Kpp + c0) * size_t(count) + size_t(i) * w + (k - c0);
}

// One general per-contingency parameter change of a line (Section 2.3):
// contingency k gives the line susceptance sus and capacity cap; z >= 0
// numbers the changes that take an AC line out (sus = 0).
struct LineChg {
  int32_t k, z;
  double sus, cap;
};

struct bf16_t {
  uint16_t u;
};

// Device control block: penalties, pending dual rescale, counters, flags.
struct alignas(16) Ctl {  // (16-byte aligned: the tape's copy kernel moves it in 16-byte words)
  double rho_p, rho_th;   // penalties used by the next iteration
  double su, sv;          // pending rescale of U (and inner duals) and of V
  double eps_eff;         // effective tolerance on the RMS residuals
  double rms_norm;        // sqrt(2 J T (K+1))
  double mu, gamma;       // adaptive penalty rule
  int32_t iter;           // iterations completed
  int32_t launches;       // finalize launches reached (completed or skipped)
  int32_t scale_iter;     // value of launches when su/sv were last set
  int32_t done;           // converged, max_iter or numeric failure
  int32_t converged;
  int32_t numeric_bad;
  int32_t adapt_every, check_every, max_iter, min_iter;
  int32_t precision;      // 0 = FP64, 1 = FP32
  int32_t cur;            // buffer holding the current iterate (0 or 1)
};
static_assert(sizeof(Ctl) % 16 == 0, "control blocks are copied in 16-byte words");

// Residual record written by the finalize kernel.
struct Rec {
  double primal_p, primal_th, dual_p, dual_th;
  double rms_primal, rms_dual, threshold, objective, rho_p, rho_th;
  int64_t iter;
  int32_t converged, precision;
};

// Precision-independent network data (device pointers into the workspace).
struct Topo {
  int32_t N, T, K, Kp, Kpp, L, G, D, B, Jnc, nR;
  const int32_t* line_from;
  const int32_t* line_to;
  const double* sus;
  const double* cap;
  const int32_t* outage_k;    // [Kpp]: line removed in contingency k, -1 none
  const int32_t* node_lptr;   // [N+1] CSR over line terminals
  const int2* node_lterm;     // (2 l + end, node at the line's other end)
  const int32_t* node_nptr;   // [N+1] CSR over generator/load/battery ids
  const int32_t* node_nterm;
  const double* deg;          // [N] terminals per node
  const double* inv_deg;      // [N] 1 / deg
  const double* hinv_sus;     // [L] 1 / (2 sus) (DC links: 1/2, unused)
  const int32_t* nc_node;     // [Jnc]
  const int32_t* ramp_idx;    // [G] index into ramp inner state, -1 = none
  const double* gen_c2;
  const double* gen_c1;
  const double* gen_pmin;     // [G][T]
  const double* gen_pmax;
  const double* gen_ramp;
  const double* load_d;       // [D][T]
  const double* bat_P;
  const double* bat_dur;
  const double* bat_eta;
  const double* bat_alpha;
  // clusters of consecutive nodes for the tiled sweep (Q = 0: not used)
  int32_t Q;
  const int32_t* clus_n0;     // [Q+1] first node of each cluster
  const int32_t* tl_ptr;      // [Q+1] range of each cluster's lines in tl
  const int4* tl;             // (line, local from node or -1, local to node or -1, far node or -1)
  const int32_t* tcsr;        // parallel to node_lterm: 2 * (index in the cluster's tl) + end
  // General line model (the sweeps run a variant that reads these only when
  // the instance has DC links or per-contingency changes)
  int32_t Ldc;
  const int32_t* line_dc;     // [L] index among the DC links, -1 for an AC line
  int32_t n_chg, Zc;          // changes; changes that take a line out
  const int32_t* chg_ptr;     // [L+1] CSR by line, entries ordered by contingency
  const LineChg* chg;
};

// Double-buffered part of the iterate.
template <typename R, typename VT>
struct Buf {
  R* P;
  R* Tm;
  VT* V1;
  VT* V2;
  R* Td;      // [T][Kpp]
  R* Hd;      // [T][chunk][Ldc][w]
  R* Tz;      // [T][Zc]
  R* U;
  R* W;
  R* TB;
};

// Iterate in one precision.  R: arithmetic/storage type, VT: storage of V.
template <typename R, typename VT>
struct State {
  Buf<R, VT> buf[2];
  R* avgW;    // [N][T]
  R* avgTB;
  R* pnc;     // [Jnc][T]
  R* thnc;
  R* vbar;
  R* ramp_st; // 4 arrays [nR][T]: beta_box, lambda_box, beta_ramp, lambda_ramp
  R* bat_st;  // 6 arrays [B][T]: beta/lambda for charge, discharge, state of charge
};

// Launch geometry and scratch shared by all kernels of one instance.
struct Geom {
  int32_t nv;             // 16-byte vectors per [Kpp] row
  int32_t n_nc_blocks;    // k_devices grid: 4 devices per block
  int32_t lanes_per_row;  // lanes per (period, node) row (power of 2, <= 64)
  int32_t rows_per_grp;   // rows per block step: 4 waves * (64 / lanes_per_row)
  int64_t n_grps;         // ceil(N*T / rows_per_grp), rows ordered t * N + n
  int32_t n_sweep_blocks; // multiple of 8
  int32_t tile_blocks;    // grid of the tiled sweep (0: node-row sweep is used)
  int32_t tile_run;       // periods per work item of the tiled sweep (a multiple of
                          // tile_group_periods; the item's cluster tables are staged once)
  int32_t n_part;         // residual partials written by the active sweep kernel
  int32_t inner_iters;
  double omega_scale;
  double* part_sweep;     // [n_sweep_blocks][5]
  double* part_nc;        // [n_nc_blocks][2]
  Ctl* ctl;
  Rec* ring;
  uint32_t* mask_rec = nullptr;  // recorded forward run: where k_devices writes
                                 // this iteration's clip masks (null: none)
};

template <typename R, typename VT>
struct KArgs {
  Topo tp;
  State<R, VT> st;
  Geom g;
};

// Work list of a batch: device-resident descriptors of every instance (an
// array of KArgs of the active precision) and prefix sums of the per-instance
// device waves and sweep row groups.
struct BatchTab {
  const void* descs;
  const int64_t* dev_prefix;  // [n_inst + 1]
  const int64_t* grp_prefix;  // [n_inst + 1]
  int32_t n_inst;
  int32_t n_sweep_blocks;
  int32_t any_gen;            // some instance has DC links or per-contingency changes
  int32_t tile_blocks;        // > 0: the tiled sweep over all instances' tiles, with this grid
  const int64_t* tile_prefix; // [n_inst + 1] prefix of the work items (runs x clusters)
  int64_t total_tiles;
  int64_t xcd_bounds[9];      // the work list split into 8 XCD ranges of equal estimated work
  int32_t* tile_queue;        // [8] items taken from each XCD range in this launch (zeroed
                              // by k_finalize_batch after every launch)
  int32_t* rescale_flag;      // set by k_finalize_batch when some instance's penalties
                              // changed, read by k_rescale_batch, cleared by the next sweep
  int64_t total_dev;
  int64_t total_grps;
};

// Host-side launchers (opf_kernels.hip).
template <typename R, typename VT>
int sweep_resident_blocks();
template <typename R, typename VT>
int tile_resident_blocks();
template <typename R, typename VT>
int tile_batch_resident_blocks();
template <typename R, typename VT>
void launch_devices(const KArgs<R, VT>& a, hipStream_t s);
template <typename R, typename VT>
void launch_sweep(const KArgs<R, VT>& a, hipStream_t s);
template <typename R, typename VT>
void launch_finalize(const KArgs<R, VT>& a, hipStream_t s);
template <typename R, typename VT>
void launch_rescale(const KArgs<R, VT>& a, hipStream_t s);
template <typename R, typename VT>
void launch_export(const KArgs<R, VT>& a, int field, double* dst, hipStream_t s);
template <typename R, typename VT>
void launch_batch_iter_devices(const BatchTab& tab, int max_T, hipStream_t s);
template <typename R, typename VT>
void launch_batch_iter_sweep(const BatchTab& tab, hipStream_t s);
template <typename R, typename VT>
void launch_batch_iter_finalize(const BatchTab& tab, hipStream_t s);
template <typename R, typename VT>
void launch_batch_iter_rescale(const BatchTab& tab, hipStream_t s);
template <typename R, typename VT>
int sweep_batch_resident_blocks();
// ---------------------------------------------------------------------------
// Reverse mode (adjoint) of unrolled iterations.  The penalty schedule of the
// forward run is held fixed; every step of an iteration is piecewise linear
// in the iterate and in the parameters (load demand, line capacity), so the
// reverse pass needs only the forward iterate at the start of each iteration
// (to recover which clips were active).

// Adjoint of the double-buffered part of the iterate (same layout as Buf).
template <typename R>
struct AdjBuf {
  R* P;
  R* Tm;
  R* V1;
  R* V2;
  R* Td;
  R* Hd;  // DC link half phase differences [T][chunk][Ldc][w] (general line model)
  R* Tz;  // half differences of lines taken out by changes [T][Zc]
  R* U;
  R* W;
  R* TB;
};

// Scalars of one recorded iteration.
struct AdjStep {
  double rp, rt;   // penalties used by the iteration
  double su, sv;   // pending ratios applied at its start (inner duals, phase duals)
  double su_next;  // ratio applied to U at its end (1 if the penalty did not change)
  int32_t last;    // 1 for the last unrolled iteration
};

template <typename R>
struct AdjArgs {
  Topo tp;
  // forward iterate at the start of the iteration (a snapshot)
  Buf<R, R> A;
  const R* avgW;
  const R* avgTB;
  const R* pnc;
  const R* thnc;
  const R* vbar;
  const R* ramp_st;
  const R* bat_st;
  // adjoint of the iterate after the iteration (read) and before it (written)
  AdjBuf<R> out, in;
  R* gsp;      // [N][T] sum over k of the node power-average adjoint (sweep -> devices)
  R* gsb;      // [N][T] same for the phase average
  R* dev_p;    // [Jnc][T] adjoint carried for the device powers
  R* dev_th;   // [Jnc][T] device phases
  R* dev_v;    // [Jnc][T] contingency-averaged device phase duals
  R* dev_x;    // [Jnc][T] adjoint of the prox target of each device
  R* dev_t;    // [Jnc][T] each device's share of the thetabar-mean adjoint
  R* ramp_adj; // adjoint of the inner state, same layout as ramp_st
  R* bat_adj;  // same for bat_st
  double* gcap;   // [T][L][Kpp] accumulated derivative w.r.t. the line capacities
  double* gload;  // [D][T] accumulated derivative w.r.t. the load demand
  double* gpmax;  // [G][T] accumulated derivative w.r.t. the generator upper limits
  const uint32_t* masks;  // clip masks the forward recorded for this iteration
  AdjStep s;
  int32_t nv, lanes_per_row, inner_iters;
  int64_t n_grps;
  double omega_scale;
  double w_obj;   // weight of the objective in the cotangent
};

// Clip masks of the time-coupled devices of one iteration, as a recorded
// forward run keeps them for the adjoint: per ramp generator r (2 bounds),
// then per battery b (3 bounds), the words [bound][through, high][e][lane]
// of its wavefront (E = slots per lane).
__host__ __device__ inline size_t mask_ramp_off(int r, int E) { return size_t(r) * 4 * E * kWave; }
__host__ __device__ inline size_t mask_bat_off(int nR, int b, int E) {
  return size_t(nR) * 4 * E * kWave + size_t(b) * 6 * E * kWave;
}
__host__ __device__ inline size_t mask_words(int nR, int B, int E) { return mask_bat_off(nR, B, E); }

// Copy of up to 20 device arrays in one launch (snapshots of the iterate).
constexpr int kMaxCopy = 20;
struct CopyList {
  const char* src[kMaxCopy];
  char* dst[kMaxCopy];
  size_t bytes[kMaxCopy];
  int32_t n;
};

template <typename R>
void launch_adj_iteration(const AdjArgs<R>& a, hipStream_t s);
template <typename R>
void launch_adj_init(const AdjArgs<R>& a, const double* cot_pnc, hipStream_t s);
template <typename R>
void launch_adj_cap(const AdjArgs<R>& a, double* grad_cap, hipStream_t s);
void launch_copy(const CopyList& cl, hipStream_t s);

// Fixed per-device workspace (opf_static.hip) of opf_load_network_static.
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
// Takes the array's device address for `device` (once; later calls return
// at once).  Must run before static_workspace(device) returns non-null.
hipError_t static_workspace_setup(int device);
void* static_workspace(int device);
// Records owner as the context whose iterate lives in the device's array and
// returns the previous one (nullptr if none); release forgets owner.
const void* static_workspace_claim(int device, const void* owner);
void static_workspace_release(int device, const void* owner);

// Widening copy of a FP32 iterate into a FP64 iterate (polishing).
template <typename VT>
void launch_widen(const KArgs<float, VT>& src, const KArgs<double, double>& dst, hipStream_t s);

}  // namespace opf
