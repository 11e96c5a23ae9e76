// HIP kernels (gfx950) of one proximal message-passing iteration for
// contingency-constrained DC OPF (arXiv 2410.17203, Section 3.2):
//
//   k_devices  step 2: prox of every generator, load and battery at the
//              contingency-averaged targets, one device per wavefront (the
//              time-coupled ones by an inner ADMM whose tridiagonal solves
//              are wavefront scans over the horizon).
//   k_sweep_tile  steps 1 and 3 fused over (period, cluster of consecutive
//              nodes) tiles staged in LDS: every line touching the cluster
//              is proxed from the previous iterate, then the node averages
//              pbar, thetabar are formed as CSR-by-node sums in a fixed order
//              (no atomics), the price u += pbar is updated, and the
//              contingency averages for step 2 and the FP64 residual partials
//              of Section 3.3 are produced.  The default.
//   k_sweep    the same per (period, node) row of contingencies and lane
//              group, for grids whose clusters cannot be built (both end
//              nodes prox a line identically, the from node stores it).
//   *_batch    the same over the instances of a batch, one launch per phase.
//   The iterate is double-buffered; the device control block says which
//   buffer is current.
//   k_finalize FP64 residual norms, the stopping test of eq. converge and the
//              adaptive penalty of Section 3.5, all on the device.
//   k_rescale  u <- (rho_old / rho_new) u after a penalty change.
//
// The path is sparse and elementwise (no dense contraction), so it runs on
// the vector ALUs and is bound by HBM bandwidth.
#include <type_traits>

#include "opf_device.h"

namespace opf {

// Step 2 for one generator, load or battery (one wavefront, all periods):
// deferred phase-dual update, theta = avg_k(thetabar - v), then the prox of
// power at target p - avg_k(pbar + u) with penalty (K+1) rho_p.  REC: also
// write the clip masks of the time-coupled prox to a.g.mask_rec (a recorded
// forward run, for the adjoint).
template <typename R, typename VT, int E, bool REC = false>
__device__ void nc_device(const KArgs<R, VT>& a, int j, int lane, R su, R sv, R rho_hat,
                          double& acc_dp, double& acc_obj) {
  const Topo& tp = a.tp;
  const int T = tp.T;
  const int n = tp.nc_node[j];
  R X[E], pold[E], pn[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    X[e] = pold[e] = pn[e] = R(0);
    if (t < T) {
      const size_t o = size_t(j) * T + t;
      const R po = a.st.pnc[o], tho = a.st.thnc[o];
      const R aw = a.st.avgW[size_t(n) * T + t], at = a.st.avgTB[size_t(n) * T + t];
      const R vb = sv * (a.st.vbar[o] + tho - at);
      a.st.vbar[o] = vb;
      a.st.thnc[o] = at - vb;
      X[e] = po - aw;
      pold[e] = po;
    }
  }
  const R omega = R(a.g.omega_scale) * rho_hat;
  double obj = 0.0;
  if (j < tp.G) {
    const int r = tp.ramp_idx[j];
    const R c2 = R(tp.gen_c2[j]), c1 = R(tp.gen_c1[j]);
    if (r < 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int t = lane * E + e;
        if (t < T)
          pn[e] = clampv(gen_target(X[e], c1, c2, rho_hat), R(tp.gen_pmin[size_t(j) * T + t]),
                         R(tp.gen_pmax[size_t(j) * T + t]));
      }
    } else if constexpr (REC) {
      ClipMasks<E, 2> mk;
      ramp_prox<R, E>(tp, a.st.ramp_st, a.st.ramp_st, r, j, X, rho_hat, omega, su, a.g.inner_iters,
                      lane, pn, mk);
      masks_store<E, 2>(a.g.mask_rec + mask_ramp_off(r, E), mk, lane);
    } else {
      NoMasks nm;
      ramp_prox<R, E>(tp, a.st.ramp_st, a.st.ramp_st, r, j, X, rho_hat, omega, su, a.g.inner_iters,
                      lane, pn, nm);
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (lane * E + e < T) obj += double(c2) * double(pn[e]) * double(pn[e]) + double(c1) * double(pn[e]);
  } else if (j < tp.G + tp.D) {
    const int d = j - tp.G;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      if (t < T) pn[e] = -R(tp.load_d[size_t(d) * T + t]);
    }
  } else if constexpr (REC) {
    const int b = j - tp.G - tp.D;
    ClipMasks<E, 3> mk;
    battery_prox<R, E>(tp, a.st.bat_st, a.st.bat_st, b, X, rho_hat, omega, su, a.g.inner_iters,
                       lane, pn, obj, mk);
    masks_store<E, 3>(a.g.mask_rec + mask_bat_off(tp.nR, b, E), mk, lane);
  } else {
    NoMasks nm;
    battery_prox<R, E>(tp, a.st.bat_st, a.st.bat_st, j - tp.G - tp.D, X, rho_hat, omega, su,
                       a.g.inner_iters, lane, pn, obj, nm);
  }
  double dp = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    if (t < T) {
      a.st.pnc[size_t(j) * T + t] = pn[e];
      const double d = double(pn[e]) - double(pold[e]);
      dp += d * d;
    }
  }
  acc_dp += double(tp.Kp) * dp;
  acc_obj += obj;
}



// Steps 1 and 3 for one (period, node) row and one 16-byte vector of
// contingencies.  acc: FP64 residual partials [sum |n| pbar^2, sum theta
// tilde^2, sum |n| dpbar^2, sum |n| dthetabar^2, sum over lines of 2 dP^2].
// GEN: the general line model (DC links, per-contingency changes); the plain
// N-1 model otherwise.  NB: line terminals per step, whose loads are all
// issued before any is used (2 pays in batches, where occupancy is already
// set by the registers; 1 for single instances).
template <typename R, typename VT, bool GEN, int NB>
__device__ inline void sweep_vec(const KArgs<R, VT>& a, const Buf<R, VT>& A, const Buf<R, VT>& B,
                                 int row, int v, int q0, int q1, bool check, R rp, R rt, R sv,
                                 double (&acc)[5], R& sumw, R& sumb) {
  constexpr int VEC = 16 / sizeof(R);
  using VR = Vec<R, VEC>;
  using VV = Vec<VT, VEC>;
  using VI = Vec<int32_t, VEC>;
  const Topo& tp = a.tp;
  const int T = tp.T;
  const int t = row / tp.N, n = row - t * tp.N;  // row = t * N + n
  const int k0 = v * VEC;
  const size_t off = ck_off(t, n, k0, tp.N, tp.Kpp);
  const VI ok = *reinterpret_cast<const VI*>(tp.outage_k + k0);
  const VR Uo = ld_stream(reinterpret_cast<const VR*>(A.U + off));
  const VR Wo = *reinterpret_cast<const VR*>(A.W + off);
  const VR Bo = *reinterpret_cast<const VR*>(A.TB + off);
  const R* td_old = A.Td + size_t(t) * tp.Kpp + k0;
  R* td_new = B.Td + size_t(t) * tp.Kpp + k0;
  // theta sums shifted by the node's first terminal phase c (for the
  // theta-tilde norm without cancellation)
  R sp[VEC], sb[VEC], c[VEC], s1[VEC], s2[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) sp[e] = sb[e] = c[e] = s1[e] = s2[e] = R(0);
  bool first = true;
  for (int q = q0; q < q1; q += NB) {
    int2 term[NB];
    VR P[NB], Tm[NB], Wx[NB], Bx[NB];
    VV V1[NB], V2[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) term[u] = (q + u < q1) ? tp.node_lterm[q + u] : make_int2(-1, 0);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (term[u].x >= 0) {
        const size_t ol = ck_off(t, term[u].x >> 1, k0, tp.L, tp.Kpp);
        const size_t oo = ck_off(t, term[u].y, k0, tp.N, tp.Kpp);
        P[u] = *reinterpret_cast<const VR*>(A.P + ol);
        Tm[u] = *reinterpret_cast<const VR*>(A.Tm + ol);
        V1[u] = *reinterpret_cast<const VV*>(A.V1 + ol);
        V2[u] = *reinterpret_cast<const VV*>(A.V2 + ol);
        Wx[u] = *reinterpret_cast<const VR*>(A.W + oo);
        Bx[u] = *reinterpret_cast<const VR*>(A.TB + oo);
      }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      if (term[u].x < 0) break;
      const int l = term[u].x >> 1;
      const bool to_end = term[u].x & 1;  // this node is the line's terminal-2 node
      const size_t ol = ck_off(t, l, k0, tp.L, tp.Kpp);
      LineOut<R, VEC> o;
      int dci = -1;
      size_t oh = 0;
      // general line model: only DC links and lines with changes need
      // per-contingency parameters; the others take the N-1 prox
      bool special = false;
      if constexpr (GEN) {
        dci = tp.line_dc[l];
        special = dci >= 0 || tp.chg_ptr[l] != tp.chg_ptr[l + 1];
      }
      if (special) {
        oh = dci >= 0 ? ck_off(t, dci, k0, tp.Ldc, tp.Kpp) : 0;
        VR Hx{};
        if (dci >= 0) Hx = *reinterpret_cast<const VR*>(A.Hd + oh);
        // (the from node stores the line, and the half differences of the
        // lines its changes take out)
        line_prox_gen<R, VT, VEC>(tp, l, k0, ok, dci, Hx, td_old, A.Tz + size_t(t) * tp.Zc,
                                  to_end ? nullptr : B.Tz + size_t(t) * tp.Zc, P[u], Tm[u],
                                  V1[u], V2[u], to_end ? Wx[u] : Wo, to_end ? Wo : Wx[u],
                                  to_end ? Bx[u] : Bo, to_end ? Bo : Bx[u], tp.Kp, rp, rt, sv, o);
      } else {
        line_prox<R, VT, VEC>(P[u], Tm[u], V1[u], V2[u], to_end ? Wx[u] : Wo,
                              to_end ? Wo : Wx[u], to_end ? Bx[u] : Bo, to_end ? Bo : Bx[u], ok, l,
                              td_old, k0, tp.Kp, R(tp.hinv_sus[l]), R(tp.cap[l]), rp, rt, sv, o);
      }
      if (!to_end) {  // the from node stores the line's new state
        VR Pn, Tn;
        VV V1n, V2n;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          Pn.x[e] = o.p[e];
          Tn.x[e] = o.tm[e];
          V1n.x[e] = DIO<VT, R>::out(o.v1[e]);
          V2n.x[e] = DIO<VT, R>::out(o.v2[e]);
          if (ok.x[e] == l) td_new[e] = o.half[e];
          if (check) {
            const double dp = double(o.p[e]) - double(P[u].x[e]);
            acc[4] += 2.0 * dp * dp;
          }
        }
        st_stream(reinterpret_cast<VR*>(B.P + ol), Pn);
        st_stream(reinterpret_cast<VR*>(B.Tm + ol), Tn);
        st_stream(reinterpret_cast<VV*>(B.V1 + ol), V1n);
        st_stream(reinterpret_cast<VV*>(B.V2 + ol), V2n);
        if (special && dci >= 0) {
          VR Hn;
#pragma unroll
          for (int e = 0; e < VEC; ++e) Hn.x[e] = o.half[e];
          *reinterpret_cast<VR*>(B.Hd + oh) = Hn;
        }
      }
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const R pj = to_end ? o.p[e] : -o.p[e];
        const R thj = to_end ? o.tm[e] - o.half[e] : o.tm[e] + o.half[e];
        sp[e] += pj;
        sb[e] += thj;
        if (first) c[e] = thj;
        const R d = thj - c[e];
        s1[e] += d;
        s2[e] += d * d;
      }
      first = false;
    }
  }
  // generators, loads, batteries: their new schedules come from k_devices
  const int r0 = tp.node_nptr[n], r1 = tp.node_nptr[n + 1];
  for (int q = r0; q < r1; ++q) {
    const int j = tp.node_nterm[q];
    const R pj = a.st.pnc[size_t(j) * T + t];
    const R thj = a.st.thnc[size_t(j) * T + t];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      sp[e] += pj;
      sb[e] += thj;
      if (first) c[e] = thj;
      const R d = thj - c[e];
      s1[e] += d;
      s2[e] += d * d;
    }
    first = false;
  }
  const double dg = tp.deg[n], idg = tp.inv_deg[n];
  const R rdg = R(dg), ridg = R(idg);
  VR Un, Wn, Bn;
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const bool valid = k0 + e < tp.Kp;
    const R pb = div_by(sp[e], rdg, ridg);
    const R tb = div_by(sb[e], rdg, ridg);
    const R un = Uo.x[e] + pb;
    const R wn = un + pb;
    if (check && valid) {
      const double dpb = double(pb);
      acc[0] += dg * dpb * dpb;
      acc[1] += fmax(double(s2[e]) - double(s1[e]) * double(s1[e]) * idg, 0.0);
      const double dd = dpb - double(Wo.x[e] - Uo.x[e]);
      acc[2] += dg * dd * dd;
      const double dt = double(tb) - double(Bo.x[e]);
      acc[3] += dg * dt * dt;
    }
    Un.x[e] = valid ? un : R(0);
    Wn.x[e] = valid ? wn : R(0);
    Bn.x[e] = valid ? tb : R(0);
    sumw += Wn.x[e];
    sumb += Bn.x[e];
  }
  st_stream(reinterpret_cast<VR*>(B.U + off), Un);
  st_stream(reinterpret_cast<VR*>(B.W + off), Wn);
  st_stream(reinterpret_cast<VR*>(B.TB + off), Bn);
}

// Rows (period, node) map onto lane groups of lanes_per_row lanes (a power
// of two, at most one wavefront); each lane takes the row's 16-byte vectors
// q, q + lanes_per_row, ...  The contingency sums of a row are reduced with
// shuffles inside its lane group (no LDS, no barrier).
template <typename R, typename VT, bool GEN>
__global__ void __launch_bounds__(kBlock) OPF_SWEEP_ATTR k_sweep(KArgs<R, VT> a) {
  Ctl* ctl = a.g.ctl;
  if (ctl->done) return;
  const int cur = ctl->cur;
  const Buf<R, VT> A = a.st.buf[cur];
  const Buf<R, VT> B = a.st.buf[cur ^ 1];
  const R rp = R(ctl->rho_p), rt = R(ctl->rho_th), sv = R(ctl->sv);
  const bool check = ((ctl->iter + 1) % ctl->check_every) == 0;
  __shared__ double sh[kBlock / kWave];
  const int lb = blockIdx.x;
  const Sweep sweep = xcd_sweep(lb, gridDim.x, a.g.n_grps);
  const int nv = a.g.nv, lpr = a.g.lanes_per_row;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int rw = lane / lpr, q = lane - rw * lpr;
  const int rows_per_wave = kWave / lpr;
  const int64_t NT = int64_t(a.tp.N) * a.tp.T;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t gi = sweep.first; gi < sweep.end; gi += sweep.step) {
    const int64_t row = (gi * (kBlock / kWave) + w) * rows_per_wave + rw;
    const bool act = row < NT;
    R sumw = R(0), sumb = R(0);
    if (act) {
      const int n = int(row) - (int(row) / a.tp.N) * a.tp.N;
      const int q0 = a.tp.node_lptr[n], q1 = a.tp.node_lptr[n + 1];
      for (int v = q; v < nv; v += lpr)
        sweep_vec<R, VT, GEN, OPF_SWEEP_BATCH>(a, A, B, int(row), v, q0, q1, check, rp, rt, sv,
                                               acc, sumw, sumb);
    }
    for (int d = lpr >> 1; d > 0; d >>= 1) {
      sumw += __shfl_xor(sumw, d);
      sumb += __shfl_xor(sumb, d);
    }
    if (act && q == 0) {
      const int t = int(row / a.tp.N), n = int(row - int64_t(t) * a.tp.N);
      a.st.avgW[size_t(n) * a.tp.T + t] = sumw / R(a.tp.Kp);
      a.st.avgTB[size_t(n) * a.tp.T + t] = sumb / R(a.tp.Kp);
    }
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double s = block_sum(acc[k], sh);
    if (threadIdx.x == 0) a.g.part_sweep[5 * lb + k] = s;
  }
}

// ---------------------------------------------------------------------------
// Tiled sweep: steps 1 and 3 for one (period, cluster of consecutive nodes)
// per workgroup, chunk by chunk of 32 contingencies.  The cluster's old W
// and thetabar rows are staged in LDS; every line touching the cluster is
// proxed once per cluster (a line with both ends inside is read and computed
// once; a line cut by the cluster boundary is computed by both clusters from
// identical inputs, the one holding its from node stores it), its new flow,
// mean phase and half phase difference are staged in LDS, and the node
// averages are then summed from LDS in the node's CSR order (no atomics).
// The running sums over contingencies for the step-2 means stay in the
// registers of the thread that owns the node across the chunks.  Tiles of
// one period follow the node order, so cut lines and far nodes read by one
// cluster were usually just read by its neighbour on the same XCD.
// One work item of the tiled sweep: cluster cq of the instance a over the
// periods [t0, t1), all contingencies; adds the item's FP64 residual
// partials to acc.  Called by the single-instance and the batched tiled
// sweeps.  The cluster's tables (its lines, terminal lists, device lists,
// degrees) are staged in LDS once for all the item's periods.  Periods are
// taken in groups: where one 128-byte pass holds all of a period's
// contingencies (K+1 <= 32 in FP32), up to tile_group_periods() periods
// share one pass, so a narrow instance fills the workgroup instead of a
// fraction of it; otherwise one period at a time, pass by pass.  Each
// thread's node rows of the next pass (or of the next group's first pass)
// are loaded while the current pass finishes.
template <typename R, typename VT, bool GEN>
__device__ __forceinline__ void tile_run(const KArgs<R, VT>& a, const Buf<R, VT>& A,
                                         const Buf<R, VT>& B, int cq, int t0, int t1, R rp, R rt,
                                         R sv, bool check, double (&acc)[5],
                                         double* item_part = nullptr) {
  constexpr int VEC = 16 / sizeof(R);
  // contingencies per pass: 128 bytes of each row (a chunk in FP32, half a
  // chunk in FP64), so that the LDS footprint is the same in both precisions
  constexpr int SUB = tile_pass_elems<R>();
  constexpr int NVMAX = SUB / VEC;  // vectors per pass row
  constexpr int NPP = sizeof(R) == 4 ? 4 : 1;
  static_assert(NVMAX <= 16 && kTileLines * NVMAX < 4096, "x / nvt by multiply and shift");
  static_assert(kTileNodes * NVMAX <= kTileBlock, "one node vector per thread and pass");
  using VR = Vec<R, VEC>;
  using VV = Vec<VT, VEC>;
  using VI = Vec<int32_t, VEC>;
  const Topo& tp = a.tp;
  __shared__ __align__(16) R sW[kTileNodes * SUB];
  __shared__ __align__(16) R sB[kTileNodes * SUB];
  __shared__ __align__(16) R sP[kTileLines * SUB];
  __shared__ __align__(16) R sTm[kTileLines * SUB];
  __shared__ __align__(16) R sH[kTileLines * SUB];
  __shared__ R sRw[kTileNodes * NVMAX], sRb[kTileNodes * NVMAX];
  __shared__ int4 sTl[kTileLines];
  // the cluster's terminal lists for the node sums, staged once per item:
  // line terminals (CSR pointers local to the cluster, entries as in tcsr)
  // and its devices (ids, and their power and phase in the group's periods;
  // at most kTileDev devices: the clusters are built so)
  __shared__ int sLp[kTileNodes + 1], sNp[kTileNodes + 1], sTc[2 * kTileLines], sJd[kTileDev];
  __shared__ R sDp[NPP * kTileDev], sDt[NPP * kTileDev];
  __shared__ float sDg[kTileNodes];  // node degrees (integers, exact)
  __shared__ double sIdg[kTileNodes];
  // running FP64 sums over a period's passes of W and thetabar per node
  // (periods with several passes are taken one at a time), kept by the
  // node's thread in LDS rather than in registers across the passes
  __shared__ double sAccW[kTileNodes], sAccB[kTileNodes];
  const int T = tp.T, N = tp.N, L = tp.L, Kpp = tp.Kpp;
  const int n0 = tp.clus_n0[cq], cn = tp.clus_n0[cq + 1] - n0;
  const int j0 = tp.tl_ptr[cq], nl = tp.tl_ptr[cq + 1] - j0;
  // general line model: which of the cluster's lines need per-contingency
  // parameters (a DC link or a line with changes), one bit per line (thread
  // j stages line j), and whether any does
  // (read after the first pass's barrier)
  static_assert(kTileLines <= kTileBlock, "one staged line per thread");
  constexpr int kSpecWords = (kTileLines + kWave - 1) / kWave;
  __shared__ uint64_t sSpec[GEN ? kSpecWords : 1];
  {
    bool sp = false;
    if (int(threadIdx.x) < nl) {
      const int4 e = tp.tl[j0 + threadIdx.x];
      sTl[threadIdx.x] = e;
      if constexpr (GEN) sp = tp.line_dc[e.x] >= 0 || tp.chg_ptr[e.x] != tp.chg_ptr[e.x + 1];
    }
    if constexpr (GEN) {
      const uint64_t m = __ballot(sp);
      if ((threadIdx.x & (kWave - 1)) == 0 && int(threadIdx.x) < kTileLines)
        sSpec[threadIdx.x / kWave] = m;
    }
  }
  const int lp0 = tp.node_lptr[n0], np0 = tp.node_nptr[n0];
  const int nlt = tp.node_lptr[n0 + cn] - lp0;  // <= 2 kTileLines (each line has two ends)
  const int ndt = tp.node_nptr[n0 + cn] - np0;  // <= kTileDev
  for (int i = threadIdx.x; i <= cn; i += kTileBlock) {
    sLp[i] = tp.node_lptr[n0 + i] - lp0;
    sNp[i] = tp.node_nptr[n0 + i] - np0;
    if (i < cn) {
      sDg[i] = float(tp.deg[n0 + i]);
      sIdg[i] = tp.inv_deg[n0 + i];
    }
  }
  for (int q = threadIdx.x; q < nlt; q += kTileBlock) sTc[q] = tp.tcsr[lp0 + q];
  for (int q = threadIdx.x; q < ndt; q += kTileBlock) sJd[q] = tp.node_nterm[np0 + q];
  const int npp = tile_group_periods<R>(Kpp);
  // Pass geometry: a pass covers the periods [tg, tg + ng) and the
  // contingencies [s0, s0 + nvc VEC) of each (one chunk or part of one).
  // Vector u of a row in the pass is period tg + u / nvc, vector u % nvc.
  // Each thread owns at most one node vector per pass.
  auto node_vec = [&](int tg, int ng, int s0) -> int64_t {
    const int c0 = s0 & ~(kChunk - 1);
    const int w = min(kChunk, Kpp - c0);
    const int nvc = min(SUB, c0 + w - s0) / VEC;
    const int nvt = ng * nvc;
    if (int(threadIdx.x) >= cn * nvt) return -1;
    const int i = int((uint32_t(threadIdx.x) * ((65536u + uint32_t(nvt) - 1u) / uint32_t(nvt))) >> 16);
    const int u = threadIdx.x - i * nvt;
    const int p = int((uint32_t(u) * ((65536u + uint32_t(nvc) - 1u) / uint32_t(nvc))) >> 16);
    const int v = u - p * nvc;
    return int64_t((size_t(tg + p) * Kpp + c0) * N + (s0 - c0) + size_t(n0 + i) * w + v * VEC);
  };
  // (held as native 16-byte vectors so that they stay in registers)
  u32x4 pW = {0u, 0u, 0u, 0u}, pB = {0u, 0u, 0u, 0u};
  {
    const int64_t o = node_vec(t0, min(npp, t1 - t0), 0);
    if (o >= 0) {
      pW = *reinterpret_cast<const u32x4*>(A.W + o);
      pB = *reinterpret_cast<const u32x4*>(A.TB + o);
    }
  }
  for (int tg = t0; tg < t1; tg += npp) {
    const int ng = min(npp, t1 - tg);  // periods in this group
    // row sums of the previous pass (ng * prev_nvc vectors per node) wait in
    // sRw, sRb; with several passes per period (then ng = 1) they are added
    // to sAccW, sAccB after the next pass's first barrier (FP64: up to 1024
    // contingencies are summed for the step-2 means)
    int prev_nvc = 0;
    for (int s0 = 0; s0 < Kpp; s0 += SUB) {
      const int c0 = s0 & ~(kChunk - 1);
      const int w = min(kChunk, Kpp - c0);                 // chunk width
      const int nvc = min(SUB, c0 + w - s0) / VEC;         // vectors per period in this pass
      const int nvt = ng * nvc;                            // vectors per row in this pass
      // x / nvt and u / nvc as a multiply and shift (exact for divisors <= 16, x < 4096)
      const uint32_t nvt_mag = (65536u + uint32_t(nvt) - 1u) / uint32_t(nvt);
      const uint32_t nvc_mag = (65536u + uint32_t(nvc) - 1u) / uint32_t(nvc);
      const bool own = int(threadIdx.x) < cn * nvt;
      const int ii = int((uint32_t(threadIdx.x) * nvt_mag) >> 16), uu = threadIdx.x - ii * nvt;
      const int pp = int((uint32_t(uu) * nvc_mag) >> 16), vv = uu - pp * nvc;
      lds_barrier();  // the previous pass's LDS is no longer read
      if (int(threadIdx.x) < cn) {  // (only this thread touches its node's entries)
        double aw = 0.0, ab = 0.0;
        if (prev_nvc > 0) {
          aw = sAccW[threadIdx.x];
          ab = sAccB[threadIdx.x];
          for (int v = 0; v < prev_nvc; ++v) {
            aw += double(sRw[threadIdx.x * prev_nvc + v]);
            ab += double(sRb[threadIdx.x * prev_nvc + v]);
          }
        }
        sAccW[threadIdx.x] = aw;
        sAccB[threadIdx.x] = ab;
      }
      if (s0 == 0) {  // device powers and phases of the group's periods
        for (int q = threadIdx.x; q < ndt * ng; q += kTileBlock) {
          const int p = q / ndt, d = q - p * ndt;
          const size_t o = size_t(sJd[d]) * T + tg + p;
          sDp[p * kTileDev + d] = a.st.pnc[o];
          sDt[p * kTileDev + d] = a.st.thnc[o];
        }
      }
      u32x4 pU = {0u, 0u, 0u, 0u};
      if (own) {
        *reinterpret_cast<u32x4*>(sW + ii * SUB + uu * VEC) = pW;
        *reinterpret_cast<u32x4*>(sB + ii * SUB + uu * VEC) = pB;
        const size_t on = (size_t(tg + pp) * Kpp + c0) * N + (s0 - c0) + size_t(n0 + ii) * w +
                          vv * VEC;
        pU = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(A.U + on));
      }
      lds_barrier();
      // One line vector of the pass: line j of the cluster, vector u of its
      // row.  SPECIAL: a line of the general line model that needs
      // per-contingency parameters (a DC link or a line with changes).  The
      // general variant takes those lines in a loop of their own, after the
      // others, so the registers of that code do not weigh on the main loop.
      auto line_item = [&](int x, auto special_tag) {
        constexpr bool SPECIAL = decltype(special_tag)::value;
        const int j = int((uint32_t(x) * nvt_mag) >> 16), u = x - j * nvt;
        const int p = int((uint32_t(u) * nvc_mag) >> 16), v = u - p * nvc;
        const int t = tg + p;
        const size_t nbase = (size_t(t) * Kpp + c0) * N + (s0 - c0);
        const size_t lbase = (size_t(t) * Kpp + c0) * L + (s0 - c0);
        const R* td_old = A.Td + size_t(t) * Kpp;
        R* td_new = B.Td + size_t(t) * Kpp;
        const int4 e = sTl[j];
        const int l = e.x;
        const int k0 = s0 + v * VEC;
        const size_t ol = lbase + size_t(l) * w + v * VEC;
        const VR P = *reinterpret_cast<const VR*>(A.P + ol);
        const VR Tm = *reinterpret_cast<const VR*>(A.Tm + ol);
        const VV V1 = *reinterpret_cast<const VV*>(A.V1 + ol);
        const VV V2 = *reinterpret_cast<const VV*>(A.V2 + ol);
        const size_t ofar = nbase + size_t(e.w < 0 ? 0 : e.w) * w + v * VEC;
        VR Wf, Wh, Bf, Bh;
        if (e.y >= 0) {
          Wf = *reinterpret_cast<const VR*>(sW + e.y * SUB + u * VEC);
          Bf = *reinterpret_cast<const VR*>(sB + e.y * SUB + u * VEC);
        } else {
          Wf = *reinterpret_cast<const VR*>(A.W + ofar);
          Bf = *reinterpret_cast<const VR*>(A.TB + ofar);
        }
        if (e.z >= 0) {
          Wh = *reinterpret_cast<const VR*>(sW + e.z * SUB + u * VEC);
          Bh = *reinterpret_cast<const VR*>(sB + e.z * SUB + u * VEC);
        } else {
          Wh = *reinterpret_cast<const VR*>(A.W + ofar);
          Bh = *reinterpret_cast<const VR*>(A.TB + ofar);
        }
        const VI ok = *reinterpret_cast<const VI*>(tp.outage_k + k0);
        LineOut<R, VEC> o;
        int dci = -1;
        size_t oh = 0;
        if constexpr (SPECIAL) {
          dci = tp.line_dc[l];
          oh = dci >= 0 ? (size_t(t) * Kpp + c0) * tp.Ldc + (s0 - c0) + size_t(dci) * w + v * VEC
                        : 0;
          VR Hx{};
          if (dci >= 0) Hx = *reinterpret_cast<const VR*>(A.Hd + oh);
          line_prox_gen<R, VT, VEC>(tp, l, k0, ok, dci, Hx, td_old + k0,
                                    A.Tz + size_t(t) * tp.Zc,
                                    e.y >= 0 ? B.Tz + size_t(t) * tp.Zc : nullptr, P, Tm, V1, V2,
                                    Wf, Wh, Bf, Bh, tp.Kp, rp, rt, sv, o);
        } else {
          line_prox<R, VT, VEC>(P, Tm, V1, V2, Wf, Wh, Bf, Bh, ok, l, td_old + k0, k0, tp.Kp,
                                R(tp.hinv_sus[l]), R(tp.cap[l]), rp, rt, sv, o);
        }
        if (e.y >= 0) {  // the cluster holding the from node stores the line
          VR Pn, Tn;
          VV V1n, V2n;
#pragma unroll
          for (int q = 0; q < VEC; ++q) {
            Pn.x[q] = o.p[q];
            Tn.x[q] = o.tm[q];
            V1n.x[q] = DIO<VT, R>::out(o.v1[q]);
            V2n.x[q] = DIO<VT, R>::out(o.v2[q]);
            if (ok.x[q] == l) td_new[k0 + q] = o.half[q];
            if (check) {
              const double dp = double(o.p[q]) - double(P.x[q]);
              acc[4] += 2.0 * dp * dp;
            }
          }
          st_stream(reinterpret_cast<VR*>(B.P + ol), Pn);
          st_stream(reinterpret_cast<VR*>(B.Tm + ol), Tn);
          st_stream(reinterpret_cast<VV*>(B.V1 + ol), V1n);
          st_stream(reinterpret_cast<VV*>(B.V2 + ol), V2n);
          if (SPECIAL && dci >= 0) {
            VR Hn;
#pragma unroll
            for (int q = 0; q < VEC; ++q) Hn.x[q] = o.half[q];
            *reinterpret_cast<VR*>(B.Hd + oh) = Hn;
          }
        }
        VR Po, To, Ho;
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          Po.x[q] = o.p[q];
          To.x[q] = o.tm[q];
          Ho.x[q] = o.half[q];
        }
        *reinterpret_cast<VR*>(sP + j * SUB + u * VEC) = Po;
        *reinterpret_cast<VR*>(sTm + j * SUB + u * VEC) = To;
        *reinterpret_cast<VR*>(sH + j * SUB + u * VEC) = Ho;
      };
      auto is_special = [&](int x) {
        const int j = int((uint32_t(x) * nvt_mag) >> 16);
        return ((sSpec[j / kWave] >> (j & (kWave - 1))) & 1ull) != 0;
      };
      bool any_spec = false;
      if constexpr (GEN) {
#pragma unroll
        for (int q = 0; q < kSpecWords; ++q) any_spec = any_spec || sSpec[q] != 0ull;
      }
      for (int x = threadIdx.x; x < nl * nvt; x += kTileBlock) {
        if constexpr (GEN) {
          if (any_spec && is_special(x)) continue;
        }
        line_item(x, std::false_type{});
      }
      if constexpr (GEN) {
        if (any_spec)
          for (int x = threadIdx.x; x < nl * nvt; x += kTileBlock)
            if (is_special(x)) line_item(x, std::true_type{});
      }
      {  // node rows of the next pass, or of the next group's first pass,
         // in flight during phase 2
        int64_t o = -1;
        if (s0 + SUB < Kpp)
          o = node_vec(tg, ng, s0 + SUB);
        else if (tg + npp < t1)
          o = node_vec(tg + npp, min(npp, t1 - tg - npp), 0);
        if (o >= 0) {
          pW = *reinterpret_cast<const u32x4*>(A.W + o);
          pB = *reinterpret_cast<const u32x4*>(A.TB + o);
        }
      }
      lds_barrier();
      if (own) {
        const int i = ii, n = n0 + i, p = pp, v = vv;
        const int k0 = s0 + v * VEC;
        const R* sdp = sDp + p * kTileDev;
        const R* sdt = sDt + p * kTileDev;
        R sp[VEC], sb[VEC], c[VEC], s1[VEC], s2[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) sp[q] = sb[q] = c[q] = s1[q] = s2[q] = R(0);
        bool first = true;
        for (int qq = sLp[i]; qq < sLp[i + 1]; ++qq) {
          const int ent = sTc[qq];
          const int j = ent >> 1;
          const bool to_end = ent & 1;
          const VR Po = *reinterpret_cast<const VR*>(sP + j * SUB + uu * VEC);
          const VR To = *reinterpret_cast<const VR*>(sTm + j * SUB + uu * VEC);
          const VR Ho = *reinterpret_cast<const VR*>(sH + j * SUB + uu * VEC);
#pragma unroll
          for (int q = 0; q < VEC; ++q) {
            const R pj = to_end ? Po.x[q] : -Po.x[q];
            const R thj = to_end ? To.x[q] - Ho.x[q] : To.x[q] + Ho.x[q];
            sp[q] += pj;
            sb[q] += thj;
            if (first) c[q] = thj;
            const R d = thj - c[q];
            s1[q] += d;
            s2[q] += d * d;
          }
          first = false;
        }
        for (int qq = sNp[i]; qq < sNp[i + 1]; ++qq) {
          const R pj = sdp[qq], thj = sdt[qq];
#pragma unroll
          for (int q = 0; q < VEC; ++q) {
            sp[q] += pj;
            sb[q] += thj;
            if (first) c[q] = thj;
            const R d = thj - c[q];
            s1[q] += d;
            s2[q] += d * d;
          }
          first = false;
        }
        const size_t on = (size_t(tg + p) * Kpp + c0) * N + (s0 - c0) + size_t(n) * w + v * VEC;
        const VR Uo = __builtin_bit_cast(VR, pU);
        const VR Wo = *reinterpret_cast<const VR*>(sW + i * SUB + uu * VEC);
        const VR Bo = *reinterpret_cast<const VR*>(sB + i * SUB + uu * VEC);
        const double dg = sDg[i], idg = sIdg[i];
        const R rdg = R(dg), ridg = R(idg);
        VR Un, Wn, Bn;
        R sumw = R(0), sumb = R(0);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          const bool valid = k0 + q < tp.Kp;
          const R pb = div_by(sp[q], rdg, ridg);
          const R tb = div_by(sb[q], rdg, ridg);
          const R un = Uo.x[q] + pb;
          const R wn = un + pb;
          if (check && valid) {
            const double dpb = double(pb);
            acc[0] += dg * dpb * dpb;
            acc[1] += fmax(double(s2[q]) - double(s1[q]) * double(s1[q]) * idg, 0.0);
            const double dd = dpb - double(Wo.x[q] - Uo.x[q]);
            acc[2] += dg * dd * dd;
            const double dt = double(tb) - double(Bo.x[q]);
            acc[3] += dg * dt * dt;
          }
          Un.x[q] = valid ? un : R(0);
          Wn.x[q] = valid ? wn : R(0);
          Bn.x[q] = valid ? tb : R(0);
          sumw += Wn.x[q];
          sumb += Bn.x[q];
        }
        st_stream(reinterpret_cast<VR*>(B.U + on), Un);
        st_stream(reinterpret_cast<VR*>(B.W + on), Wn);
        st_stream(reinterpret_cast<VR*>(B.TB + on), Bn);
        // row sums indexed (node, period, vector): ii * nvt + uu
        sRw[threadIdx.x] = sumw;
        sRb[threadIdx.x] = sumb;
      }
      prev_nvc = nvc;
    }
    lds_barrier();
    if (int(threadIdx.x) < cn * ng) {
      const int i = int(threadIdx.x) / ng, p = int(threadIdx.x) - i * ng;
      // (sAcc holds the earlier passes of a period taken in several passes,
      // and zero otherwise)
      double aw = ng == 1 ? sAccW[i] : 0.0, ab = ng == 1 ? sAccB[i] : 0.0;
      for (int v = 0; v < prev_nvc; ++v) {
        aw += double(sRw[(i * ng + p) * prev_nvc + v]);
        ab += double(sRb[(i * ng + p) * prev_nvc + v]);
      }
      const size_t o = size_t(n0 + i) * T + tg + p;
      a.st.avgW[o] = R(aw / double(tp.Kp));
      a.st.avgTB[o] = R(ab / double(tp.Kp));
    }
  }
  if (item_part) {  // this item's residual partials: each wave's sums, then the waves in order
    // (in sP, whose last reads were in the node phase, before the barrier above)
    constexpr int kWaves = kTileBlock / kWave;
    static_assert(5 * kWaves * sizeof(double) <= sizeof(sP), "wave sums fit in sP");
    double* const scr = reinterpret_cast<double*>(sP);
    double ws[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      ws[k] = wave_sum(acc[k]);
      acc[k] = 0.0;
    }
    if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
      for (int k = 0; k < 5; ++k) scr[(threadIdx.x / kWave) * 5 + k] = ws[k];
    lds_barrier();
    if (threadIdx.x < 5) {
      double v = 0.0;
      for (int w = 0; w < kWaves; ++w) v += scr[w * 5 + threadIdx.x];
      item_part[threadIdx.x] = v;
    }
  }
}

// (4 waves per SIMD: two workgroups per CU, the most its LDS footprint allows)
template <typename R, typename VT, bool GEN>
__global__ void __launch_bounds__(kTileBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_sweep_tile(KArgs<R, VT> a) {
  Ctl* ctl = a.g.ctl;
  if (ctl->done) return;
  const Topo& tp = a.tp;
  const int cur = ctl->cur;
  const Buf<R, VT> A = a.st.buf[cur];
  const Buf<R, VT> B = a.st.buf[cur ^ 1];
  const R rp = R(ctl->rho_p), rt = R(ctl->rho_th), sv = R(ctl->sv);
  const bool check = ((ctl->iter + 1) % ctl->check_every) == 0;
  __shared__ double sh[kTileBlock / kWave];
  // work items: (run of tile_run periods, cluster), clusters innermost
  const int run = a.g.tile_run;
  const int64_t n_items = int64_t((tp.T + run - 1) / run) * tp.Q;
  const Sweep sweep = xcd_sweep(blockIdx.x, gridDim.x, n_items);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t item = sweep.first; item < sweep.end; item += sweep.step) {
    const int r = int(item / tp.Q), cq = int(item - int64_t(r) * tp.Q);
    const int t0 = r * run;
    tile_run<R, VT, GEN>(a, A, B, cq, t0, min(tp.T, t0 + run), rp, rt, sv, check, acc);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double s = block_sum<kTileBlock>(acc[k], sh);
    if (threadIdx.x == 0) a.g.part_sweep[5 * blockIdx.x + k] = s;
  }
}

// Step 2 for all generators, loads and batteries, one per wavefront.
template <typename R, typename VT, int E, bool REC>
__global__ void __launch_bounds__(kBlock) k_devices(KArgs<R, VT> a) {
  Ctl* ctl = a.g.ctl;
  if (ctl->done) return;
  const R rp = R(ctl->rho_p), su = R(ctl->su), sv = R(ctl->sv);
  __shared__ double sh[kBlock / kWave];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * (kBlock / kWave) + w;
  double dp = 0.0, ob = 0.0;
  if (j < a.tp.Jnc) nc_device<R, VT, E, REC>(a, j, lane, su, sv, R(a.tp.Kp) * rp, dp, ob);
  dp = block_sum(dp, sh);
  ob = block_sum(ob, sh);
  if (threadIdx.x == 0) {
    a.g.part_nc[2 * blockIdx.x] = dp;
    a.g.part_nc[2 * blockIdx.x + 1] = ob;
  }
}

// ---------------------------------------------------------------------------
// Residual norms, stopping test and adaptive penalty (single block).
__device__ inline double adapt_rule(double rho, double rpri, double rdual, double mu, double gamma) {
  if (rpri > mu * rdual) return rho * gamma;
  if (rdual > mu * rpri) return rho / gamma;
  return rho;
}

// Residual norms, stopping test and adaptive penalty of one instance, run by
// one block.  Partials: n_sweep entries of 5 sums, n_nc entries of 2.
template <typename R, typename VT>
__device__ void finalize_body(const KArgs<R, VT>& a, int n_sweep, int n_nc) {
  Ctl* ctl = a.g.ctl;
  __shared__ double sh[kBlock / kWave];
  __shared__ int sdone;
  if (threadIdx.x == 0) sdone = ctl->done;
  __syncthreads();
  if (sdone) {
    if (threadIdx.x == 0) ctl->launches += 1;
    return;
  }
  const int iter = ctl->iter + 1;
  const bool check = (iter % ctl->check_every) == 0;
  double s[7] = {0, 0, 0, 0, 0, 0, 0};  // 5 sweep partials, device dual, objective
  if (check) {
    for (int i = threadIdx.x; i < n_sweep; i += kBlock)
#pragma unroll
      for (int k = 0; k < 5; ++k) s[k] += a.g.part_sweep[5 * i + k];
    for (int i = threadIdx.x; i < n_nc; i += kBlock) {
      s[5] += a.g.part_nc[2 * i];
      s[6] += a.g.part_nc[2 * i + 1];
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) s[k] = block_sum(s[k], sh);
  }
  if (threadIdx.x != 0) return;
  const double rp = ctl->rho_p, rt = ctl->rho_th;
  double su = 1.0, sv = 1.0;
  int conv = 0, bad = 0;
  if (check) {
    // a NaN or infinite partial (an overflowed or NaN iterate) is a numeric
    // failure; it must be caught before the fmax clamps below, which would
    // turn a NaN into 0
    bool parts_ok = true;
#pragma unroll
    for (int k = 0; k < 7; ++k) parts_ok = parts_ok && isfinite(s[k]);
    // ||ptilde' - ptilde||^2 = sum over terminal copies of dp^2 - sum |n| dpbar^2
    const double pp = fmax(s[0], 0.0), pt = fmax(s[1], 0.0);
    const double dp = rp * rp * fmax(s[4] + s[5] - s[2], 0.0);
    const double dt = rt * rt * fmax(s[3], 0.0);
    Rec rec;
    rec.primal_p = sqrt(pp);
    rec.primal_th = sqrt(pt);
    rec.dual_p = sqrt(dp);
    rec.dual_th = sqrt(dt);
    rec.rms_primal = sqrt(pp + pt) / ctl->rms_norm;
    rec.rms_dual = sqrt(dp + dt) / ctl->rms_norm;
    rec.threshold = ctl->eps_eff;
    rec.objective = s[6];
    rec.rho_p = rp;
    rec.rho_th = rt;
    rec.iter = iter;
    rec.precision = ctl->precision;
    bad = !(parts_ok && isfinite(rec.rms_primal) && isfinite(rec.rms_dual));
    conv = !bad && fmax(rec.rms_primal, rec.rms_dual) <= ctl->eps_eff && iter >= ctl->min_iter;
    rec.converged = conv;
    if (ctl->adapt_every > 0 && iter % ctl->adapt_every == 0 && !bad) {
      const double np = adapt_rule(rp, rec.primal_p, rec.dual_p, ctl->mu, ctl->gamma);
      const double nt = adapt_rule(rt, rec.primal_th, rec.dual_th, ctl->mu, ctl->gamma);
      su = rp / np;
      sv = rt / nt;
      ctl->rho_p = np;
      ctl->rho_th = nt;
    }
    a.g.ring[(iter - 1) % kRing] = rec;
  }
  ctl->su = su;
  ctl->sv = sv;
  ctl->launches += 1;
  ctl->scale_iter = ctl->launches;
  ctl->iter = iter;
  ctl->cur ^= 1;  // the sweep wrote the other buffer
  if (conv) ctl->converged = 1;
  if (bad) ctl->numeric_bad = 1;
  if (conv || bad || iter >= ctl->max_iter) ctl->done = 1;
}

template <typename R, typename VT>
__global__ void __launch_bounds__(kBlock) k_finalize(KArgs<R, VT> a) {
  finalize_body(a, a.g.n_part, a.g.n_nc_blocks);
}

// u <- su u after a penalty change for one (period, node) row of the current
// buffer (lane group of lanes_per_row lanes).
template <typename R, typename VT>
__device__ inline void rescale_row(const KArgs<R, VT>& a, const Buf<R, VT>& C, R su, int64_t row,
                                   int q, int lpr) {
  constexpr int VEC = 16 / sizeof(R);
  using VR = Vec<R, VEC>;
  const int64_t NT = int64_t(a.tp.N) * a.tp.T;
  const bool act = row < NT;
  R sumw = R(0);
  if (act) {
    for (int v = q; v < a.g.nv; v += lpr) {
      const int t = int(row / a.tp.N), n = int(row - int64_t(t) * a.tp.N);
      const size_t off = ck_off(t, n, v * VEC, a.tp.N, a.tp.Kpp);
      const VR U = *reinterpret_cast<const VR*>(C.U + off);
      const VR W = *reinterpret_cast<const VR*>(C.W + off);
      VR Un, Wn;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        Un.x[e] = su * U.x[e];
        Wn.x[e] = W.x[e] + (su - R(1)) * U.x[e];
        sumw += Wn.x[e];
      }
      *reinterpret_cast<VR*>(C.U + off) = Un;
      *reinterpret_cast<VR*>(C.W + off) = Wn;
    }
  }
  for (int d = lpr >> 1; d > 0; d >>= 1) sumw += __shfl_xor(sumw, d);
  if (act && q == 0) {
    const int t = int(row / a.tp.N), n = int(row - int64_t(t) * a.tp.N);
    a.st.avgW[size_t(n) * a.tp.T + t] = sumw / R(a.tp.Kp);
  }
}

template <typename R, typename VT>
__global__ void __launch_bounds__(kBlock) k_rescale(KArgs<R, VT> a) {
  Ctl* ctl = a.g.ctl;
  if (ctl->scale_iter != ctl->launches) return;
  const R su = R(ctl->su);
  if (su == R(1)) return;
  const Buf<R, VT> C = a.st.buf[ctl->cur];
  const Sweep sweep = xcd_sweep(blockIdx.x, gridDim.x, a.g.n_grps);
  const int lpr = a.g.lanes_per_row;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int rw = lane / lpr, q = lane - rw * lpr;
  const int rows_per_wave = kWave / lpr;
  for (int64_t gi = sweep.first; gi < sweep.end; gi += sweep.step)
    rescale_row(a, C, su, (gi * (kBlock / kWave) + w) * rows_per_wave + rw, q, lpr);
}

// ---------------------------------------------------------------------------
// Batched execution: many instances of uneven size, one launch per phase over
// a work list spanning all of them.  Each instance keeps its own control
// block (penalties, counters, convergence) and buffers; finished instances
// are skipped.  Residual partials are written per (row group, wave) and per
// device, so no block-wide barrier is needed inside the work loops.
//
// The instances' descriptors are read through the constant address space
// (the host writes them; no kernel does).  Pointers loaded from constant
// memory are taken by the compiler to address global memory, so each
// instance's state is accessed with global loads and stores as in the
// single-instance kernels, whose arguments are constant too.  Read through a
// generic pointer they would be flat accesses, which also count against the
// LDS wait counter: every LDS barrier of the tiled sweep would then wait for
// all of the workgroup's HBM loads in flight.
template <typename R, typename VT>
struct BatchDescs {
  using CA = __attribute__((address_space(4))) const KArgs<R, VT>;
  const CA* p;
  __device__ explicit BatchDescs(const void* d) : p((const CA*)d) {}
  // a copy of instance i's descriptor (its fields live in scalar registers)
  __device__ KArgs<R, VT> operator[](int i) const { return *(const KArgs<R, VT>*)(p + i); }
  // buffer k of instance i (k need not be known at compile time)
  __device__ Buf<R, VT> buf(int i, int k) const {
    return *(const Buf<R, VT>*)(&p[i].st.buf[k]);
  }
  __device__ Ctl* ctl(int i) const { return p[i].g.ctl; }
};

__device__ inline int find_inst(const int64_t* prefix, int n, int64_t g) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <typename R, typename VT, int E>
__global__ void __launch_bounds__(kBlock) k_devices_batch(BatchTab tab) {
  const BatchDescs<R, VT> descs(tab.descs);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t gw = int64_t(blockIdx.x) * (kBlock / kWave) + w;
  if (gw >= tab.total_dev) return;
  const int i = find_inst(tab.dev_prefix, tab.n_inst, gw);
  const KArgs<R, VT> a = descs[i];
  Ctl* ctl = a.g.ctl;
  if (ctl->done) return;
  const int j = int(gw - tab.dev_prefix[i]);
  const R rp = R(ctl->rho_p), su = R(ctl->su), sv = R(ctl->sv);
  double dp = 0.0, ob = 0.0;
  nc_device<R, VT, E>(a, j, lane, su, sv, R(a.tp.Kp) * rp, dp, ob);
  dp = wave_sum(dp);
  ob = wave_sum(ob);
  if (lane == 0) {
    a.g.part_nc[2 * j] = dp;
    a.g.part_nc[2 * j + 1] = ob;
  }
}

template <typename R, typename VT, bool GEN>
__global__ void __launch_bounds__(kBlock) k_sweep_batch(BatchTab tab) {
  const BatchDescs<R, VT> descs(tab.descs);
  if (blockIdx.x == 0 && threadIdx.x == 0) *tab.rescale_flag = 0;  // (set by the finalize after)
  const Sweep sweep = xcd_sweep(blockIdx.x, gridDim.x, tab.total_grps);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int64_t gi = sweep.first; gi < sweep.end; gi += sweep.step) {
    const int i = find_inst(tab.grp_prefix, tab.n_inst, gi);
    const KArgs<R, VT> a = descs[i];
    Ctl* ctl = a.g.ctl;
    if (ctl->done) continue;
    const int cur = ctl->cur;
    const Buf<R, VT> A = descs.buf(i, cur);
    const Buf<R, VT> B = descs.buf(i, cur ^ 1);
    const R rp = R(ctl->rho_p), rt = R(ctl->rho_th), sv = R(ctl->sv);
    const bool check = ((ctl->iter + 1) % ctl->check_every) == 0;
    const int64_t li = gi - tab.grp_prefix[i];
    const int nv = a.g.nv, lpr = a.g.lanes_per_row;
    const int rw = lane / lpr, q = lane - rw * lpr;
    const int64_t row = (li * (kBlock / kWave) + w) * (kWave / lpr) + rw;
    const int64_t NT = int64_t(a.tp.N) * a.tp.T;
    const bool act = row < NT;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    R sumw = R(0), sumb = R(0);
    if (act) {
      const int n = int(row) - (int(row) / a.tp.N) * a.tp.N;
      const int q0 = a.tp.node_lptr[n], q1 = a.tp.node_lptr[n + 1];
      for (int v = q; v < nv; v += lpr)
        sweep_vec<R, VT, GEN, 2>(a, A, B, int(row), v, q0, q1, check, rp, rt, sv, acc, sumw, sumb);
    }
    for (int d = lpr >> 1; d > 0; d >>= 1) {
      sumw += __shfl_xor(sumw, d);
      sumb += __shfl_xor(sumb, d);
    }
    if (act && q == 0) {
      const int t = int(row / a.tp.N), n = int(row - int64_t(t) * a.tp.N);
      a.st.avgW[size_t(n) * a.tp.T + t] = sumw / R(a.tp.Kp);
      a.st.avgTB[size_t(n) * a.tp.T + t] = sumb / R(a.tp.Kp);
    }
    if (check) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) a.g.part_sweep[5 * (li * (kBlock / kWave) + w) + k] = s;
      }
    }
  }
}

// Tiled sweep over the work items of all instances of a batch (one work
// list, in instance order).  Items are handed out as the workgroups free
// up: each XCD's range of the list (split by estimated work) has a counter,
// a workgroup takes the next item of its own XCD's range and, once that
// range is used up, of the other ranges in turn, so the workgroups finish
// together whatever the sizes of their items.  An item writes its own FP64
// residual partials (each wave's sums, then the waves in order) to its
// instance's slot for that item, so the reduction order does not depend on
// which workgroup ran the item.  The counters are reset to zero by
// k_finalize_batch, which follows every launch of this kernel.
template <typename R, typename VT, bool GEN>
__global__ void __launch_bounds__(kTileBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_sweep_tile_batch(BatchTab tab) {
  const BatchDescs<R, VT> descs(tab.descs);
  if (blockIdx.x == 0 && threadIdx.x == 0) *tab.rescale_flag = 0;  // (set by the finalize after)
  __shared__ int64_t sItem[2];  // the next item, double-buffered by parity
  const int x0 = blockIdx.x & 7;
  int xs = 0;  // (thread 0) ranges used up so far, own range first
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int n = 0;; ++n) {
    if (threadIdx.x == 0) {
      int64_t g = -1;
      for (; xs < 8; ++xs) {
        const int x = (x0 + xs) & 7;
        const int64_t c = tab.xcd_bounds[x] + int64_t(atomicAdd(tab.tile_queue + x, 1));
        if (c < tab.xcd_bounds[x + 1]) {
          g = c;
          break;
        }
      }
      sItem[n & 1] = g;
    }
    lds_barrier();
    // (the same value in every lane: made a scalar so that the instance's
    // descriptor is read through the scalar unit, as with a computed index)
    const int64_t gl = sItem[n & 1];
    const int64_t g = int64_t(
        (uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(uint64_t(gl) >> 32)))) << 32) |
        uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(uint64_t(gl)))))));
    if (g < 0) break;
    const int i = find_inst(tab.tile_prefix, tab.n_inst, g);
    if (descs.ctl(i)->done) {
      // a stopped instance: its remaining items in this range are skipped at once
      if (threadIdx.x == 0) {
        const int x = (x0 + xs) & 7;
        const int64_t b = tab.xcd_bounds[x], e = tab.xcd_bounds[x + 1];
        atomicMax(tab.tile_queue + x, int(min(e, tab.tile_prefix[i + 1]) - b));
      }
      continue;
    }
    const KArgs<R, VT> a = descs[i];
    Ctl* ctl = a.g.ctl;
    const int cur = ctl->cur;
    const R rp = R(ctl->rho_p), rt = R(ctl->rho_th), sv = R(ctl->sv);
    const bool check = ((ctl->iter + 1) % ctl->check_every) == 0;
    const int64_t li = g - tab.tile_prefix[i];
    const int r = int(li / a.tp.Q), cq = int(li - int64_t(r) * a.tp.Q);
    const int t0 = r * a.g.tile_run;
    tile_run<R, VT, GEN>(a, descs.buf(i, cur), descs.buf(i, cur ^ 1), cq, t0,
                         min(a.tp.T, t0 + a.g.tile_run), rp, rt, sv, check, acc,
                         check ? a.g.part_sweep + 5 * li : nullptr);
  }
}

template <typename R, typename VT>
__global__ void __launch_bounds__(kBlock) k_finalize_batch(BatchTab tab) {
  const KArgs<R, VT> a = BatchDescs<R, VT>(tab.descs)[blockIdx.x];
  // the tiled sweep's work counters start the next launch at zero
  if (blockIdx.x == 0 && threadIdx.x < 8) tab.tile_queue[threadIdx.x] = 0;
  const int64_t ng = tab.grp_prefix[blockIdx.x + 1] - tab.grp_prefix[blockIdx.x];
  // partials: one per work item of the tiled sweep, else per (row group, wavefront)
  const int64_t n_items = tab.tile_prefix[blockIdx.x + 1] - tab.tile_prefix[blockIdx.x];
  const int n_sweep = tab.tile_blocks > 0 ? int(n_items) : int(ng * (kBlock / kWave));
  finalize_body(a, n_sweep, a.tp.Jnc);
  // (thread 0 has just set the control block: a penalty change to apply)
  if (threadIdx.x == 0 && a.g.ctl->scale_iter == a.g.ctl->launches && a.g.ctl->su != 1.0)
    *tab.rescale_flag = 1;
}

template <typename R, typename VT>
__global__ void __launch_bounds__(kBlock) k_rescale_batch(BatchTab tab) {
  if (*tab.rescale_flag == 0) return;  // no instance changed its penalties
  const BatchDescs<R, VT> descs(tab.descs);
  const Sweep sweep = xcd_sweep(blockIdx.x, gridDim.x, tab.total_grps);
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  // (the block's row groups ascend, so each instance is looked up once, and
  // an instance without a penalty change is passed over in one step)
  for (int64_t gi = sweep.first; gi < sweep.end;) {
    const int i = find_inst(tab.grp_prefix, tab.n_inst, gi);
    const int64_t gend = min(tab.grp_prefix[i + 1], sweep.end);
    const KArgs<R, VT> a = descs[i];
    Ctl* ctl = a.g.ctl;
    const R su = R(ctl->su);
    const bool act = ctl->scale_iter == ctl->launches && su != R(1);
    if (act) {
      const int lpr = a.g.lanes_per_row;
      const int rw = lane / lpr, q = lane - rw * lpr;
      const Buf<R, VT> C = descs.buf(i, ctl->cur);
      for (; gi < gend; gi += sweep.step) {
        const int64_t li = gi - tab.grp_prefix[i];
        rescale_row(a, C, su, (li * (kBlock / kWave) + w) * (kWave / lpr) + rw, q, lpr);
      }
    } else {
      gi += (gend - gi + sweep.step - 1) / sweep.step * sweep.step;  // first one >= gend
    }
  }
}

// ---------------------------------------------------------------------------
// Export of one field of the iterate in the paper's layout, as FP64.
template <typename R, typename VT>
__global__ void __launch_bounds__(kBlock) k_export(KArgs<R, VT> a, int field, double* dst,
                                                   int64_t count) {
  const Topo& tp = a.tp;
  const double sv = a.g.ctl->sv;
  const Buf<R, VT> C = a.st.buf[a.g.ctl->cur];
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= count) return;
  const int T = tp.T;
  if (field <= 4) {  // [Kp][L][T]
    const int t = int(i % T);
    const int l = int((i / T) % tp.L);
    const int k = int(i / (int64_t(T) * tp.L));
    const size_t o = ck_off(t, l, k, tp.L, tp.Kpp);
    const double P = double(C.P[o]);
    if (field == 0) {
      dst[i] = P;
      return;
    }
    const bool outg = tp.outage_k[k] == l;
    const int dci = tp.line_dc[l];
    double half;
    if (dci >= 0) {
      half = double(C.Hd[ck_off(t, dci, k, tp.Ldc, tp.Kpp)]);
    } else if (outg) {
      half = double(C.Td[size_t(t) * tp.Kpp + k]);
    } else {
      double s = tp.sus[l];
      int z = -1;
      for (int c = tp.chg_ptr[l]; c < tp.chg_ptr[l + 1]; ++c)
        if (tp.chg[c].k == k) {
          s = tp.chg[c].sus;
          z = tp.chg[c].z;
        }
      half = z >= 0 ? double(C.Tz[size_t(t) * tp.Zc + z]) : P * (0.5 / s);
    }
    const double th1 = double(C.Tm[o]) + half, th2 = double(C.Tm[o]) - half;
    if (field == 1) dst[i] = th1;
    if (field == 2) dst[i] = th2;
    if (field == 3 || field == 4) {
      const int nd = field == 3 ? tp.line_from[l] : tp.line_to[l];
      const double tb = double(C.TB[ck_off(t, nd, k, tp.N, tp.Kpp)]);
      const double vs = double(DIO<VT, R>::in(field == 3 ? C.V1[o] : C.V2[o]));
      dst[i] = sv * (vs + (field == 3 ? th1 : th2) - tb);
    }
    return;
  }
  if (field <= 7) {  // [Kp][N][T]
    const int t = int(i % T);
    const int n = int((i / T) % tp.N);
    const int k = int(i / (int64_t(T) * tp.N));
    const size_t o = ck_off(t, n, k, tp.N, tp.Kpp);
    if (field == 5) dst[i] = double(C.U[o]);
    if (field == 6) dst[i] = double(C.W[o]) - double(C.U[o]);
    if (field == 7) dst[i] = double(C.TB[o]);
    return;
  }
  // [Jnc][T]
  const int t = int(i % T);
  const int j = int(i / T);
  if (field == 8) dst[i] = double(a.st.pnc[i]);
  if (field == 9) dst[i] = double(a.st.thnc[i]);
  if (field == 10) {
    const int n = tp.nc_node[j];
    dst[i] = sv * (double(a.st.vbar[i]) + double(a.st.thnc[i]) - double(a.st.avgTB[size_t(n) * T + t]));
  }
}

// Widening copy (FP32 iterate -> FP64 iterate); same element layout.
template <typename S, typename D>
__global__ void __launch_bounds__(kBlock) k_widen(const S* src, D* dst, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) dst[i] = D(DIO<S, float>::in(src[i]));
}

// ---------------------------------------------------------------------------
// Host launchers.

template <typename R, typename VT>
void launch_devices(const KArgs<R, VT>& a, hipStream_t s) {
  if (a.g.n_nc_blocks == 0) return;
  const int E = (a.tp.T + kWave - 1) / kWave;
  const dim3 grid(a.g.n_nc_blocks);
  if (a.g.mask_rec) {
    switch (E) {
      case 1: k_devices<R, VT, 1, true><<<grid, kBlock, 0, s>>>(a); break;
      case 2: k_devices<R, VT, 2, true><<<grid, kBlock, 0, s>>>(a); break;
      case 3: k_devices<R, VT, 3, true><<<grid, kBlock, 0, s>>>(a); break;
      default: k_devices<R, VT, 4, true><<<grid, kBlock, 0, s>>>(a); break;
    }
    return;
  }
  switch (E) {
    case 1: k_devices<R, VT, 1, false><<<grid, kBlock, 0, s>>>(a); break;
    case 2: k_devices<R, VT, 2, false><<<grid, kBlock, 0, s>>>(a); break;
    case 3: k_devices<R, VT, 3, false><<<grid, kBlock, 0, s>>>(a); break;
    default: k_devices<R, VT, 4, false><<<grid, kBlock, 0, s>>>(a); break;
  }
}

// Blocks of k_sweep that are resident at once on the current device: the
// sweep grid is sized to this so that all blocks advance as one front.
template <typename R, typename VT>
int sweep_resident_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep<R, VT, false>, kBlock, 0) != hipSuccess)
    return 0;
  return cus * per;
}

template <typename R, typename VT>
void launch_sweep(const KArgs<R, VT>& a, hipStream_t s) {
  const bool gen = a.tp.Ldc > 0 || a.tp.n_chg > 0;
  if (a.g.tile_blocks > 0) {
    if (gen)
      k_sweep_tile<R, VT, true><<<a.g.tile_blocks, kTileBlock, 0, s>>>(a);
    else
      k_sweep_tile<R, VT, false><<<a.g.tile_blocks, kTileBlock, 0, s>>>(a);
  } else {
    if (gen)
      k_sweep<R, VT, true><<<a.g.n_sweep_blocks, kBlock, 0, s>>>(a);
    else
      k_sweep<R, VT, false><<<a.g.n_sweep_blocks, kBlock, 0, s>>>(a);
  }
}

// Blocks of the tiled sweep resident at once on the current device.
template <typename R, typename VT>
int tile_resident_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep_tile<R, VT, false>, kTileBlock, 0) !=
      hipSuccess)
    return 0;
  return cus * per;
}

template <typename R, typename VT>
int tile_batch_resident_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep_tile_batch<R, VT, false>,
                                                   kTileBlock, 0) != hipSuccess)
    return 0;
  return cus * per;
}

template <typename R, typename VT>
void launch_finalize(const KArgs<R, VT>& a, hipStream_t s) {
  k_finalize<R, VT><<<1, kBlock, 0, s>>>(a);
}

template <typename R, typename VT>
void launch_rescale(const KArgs<R, VT>& a, hipStream_t s) {
  k_rescale<R, VT><<<a.g.n_sweep_blocks, kBlock, 0, s>>>(a);
}

template <typename R, typename VT>
void launch_export(const KArgs<R, VT>& a, int field, double* dst, hipStream_t s) {
  int64_t count;
  const int64_t KT = int64_t(a.tp.Kp) * a.tp.T;
  if (field <= 4)
    count = KT * a.tp.L;
  else if (field <= 7)
    count = KT * a.tp.N;
  else
    count = int64_t(a.tp.Jnc) * a.tp.T;
  if (count == 0) return;
  const int64_t grid = (count + kBlock - 1) / kBlock;
  k_export<R, VT><<<dim3(unsigned(grid)), kBlock, 0, s>>>(a, field, dst, count);
}

template <typename S, typename D>
static void widen(const S* src, D* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_widen<S, D><<<dim3(unsigned((n + kBlock - 1) / kBlock)), kBlock, 0, s>>>(src, dst, n);
}

template <typename VT>
void launch_widen(const KArgs<float, VT>& a, const KArgs<double, double>& b, hipStream_t s) {
  const Topo& tp = a.tp;
  const int64_t line = int64_t(tp.L) * tp.T * tp.Kpp;
  const int64_t node = int64_t(tp.N) * tp.T * tp.Kpp;
  for (int i = 0; i < 2; ++i) {
    const Buf<float, VT>& x = a.st.buf[i];
    const Buf<double, double>& y = b.st.buf[i];
    widen(x.P, y.P, line, s);
    widen(x.Tm, y.Tm, line, s);
    widen(x.V1, y.V1, line, s);
    widen(x.V2, y.V2, line, s);
    widen(x.Td, y.Td, int64_t(tp.T) * tp.Kpp, s);
    widen(x.Hd, y.Hd, int64_t(tp.Ldc) * tp.T * tp.Kpp, s);
    widen(x.Tz, y.Tz, int64_t(tp.T) * tp.Zc, s);
    widen(x.U, y.U, node, s);
    widen(x.W, y.W, node, s);
    widen(x.TB, y.TB, node, s);
  }
  widen(a.st.avgW, b.st.avgW, int64_t(tp.N) * tp.T, s);
  widen(a.st.avgTB, b.st.avgTB, int64_t(tp.N) * tp.T, s);
  const int64_t nc = int64_t(tp.Jnc) * tp.T;
  widen(a.st.pnc, b.st.pnc, nc, s);
  widen(a.st.thnc, b.st.thnc, nc, s);
  widen(a.st.vbar, b.st.vbar, nc, s);
  widen(a.st.ramp_st, b.st.ramp_st, 4 * int64_t(tp.nR) * tp.T, s);
  widen(a.st.bat_st, b.st.bat_st, 6 * int64_t(tp.B) * tp.T, s);
}

template <typename R, typename VT>
void launch_batch_iter_devices(const BatchTab& tab, int max_T, hipStream_t s) {
  const int64_t grid = (tab.total_dev + (kBlock / kWave) - 1) / (kBlock / kWave);
  if (grid == 0) return;
  const int E = (max_T + kWave - 1) / kWave;
  switch (E) {
    case 1: k_devices_batch<R, VT, 1><<<dim3(unsigned(grid)), kBlock, 0, s>>>(tab); break;
    case 2: k_devices_batch<R, VT, 2><<<dim3(unsigned(grid)), kBlock, 0, s>>>(tab); break;
    case 3: k_devices_batch<R, VT, 3><<<dim3(unsigned(grid)), kBlock, 0, s>>>(tab); break;
    default: k_devices_batch<R, VT, 4><<<dim3(unsigned(grid)), kBlock, 0, s>>>(tab); break;
  }
}

template <typename R, typename VT>
void launch_batch_iter_sweep(const BatchTab& tab, hipStream_t s) {
  if (tab.tile_blocks > 0) {
    if (tab.any_gen)
      k_sweep_tile_batch<R, VT, true><<<tab.tile_blocks, kTileBlock, 0, s>>>(tab);
    else
      k_sweep_tile_batch<R, VT, false><<<tab.tile_blocks, kTileBlock, 0, s>>>(tab);
  } else if (tab.any_gen) {
    k_sweep_batch<R, VT, true><<<tab.n_sweep_blocks, kBlock, 0, s>>>(tab);
  } else {
    k_sweep_batch<R, VT, false><<<tab.n_sweep_blocks, kBlock, 0, s>>>(tab);
  }
}

template <typename R, typename VT>
void launch_batch_iter_finalize(const BatchTab& tab, hipStream_t s) {
  k_finalize_batch<R, VT><<<tab.n_inst, kBlock, 0, s>>>(tab);
}

template <typename R, typename VT>
void launch_batch_iter_rescale(const BatchTab& tab, hipStream_t s) {
  k_rescale_batch<R, VT><<<tab.n_sweep_blocks, kBlock, 0, s>>>(tab);
}

template <typename R, typename VT>
int sweep_batch_resident_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sweep_batch<R, VT, false>, kBlock, 0) != hipSuccess)
    return 0;
  return cus * per;
}

#define OPF_INSTANTIATE(R, VT)                                                       \
  template void launch_batch_iter_devices<R, VT>(const BatchTab&, int, hipStream_t); \
  template void launch_batch_iter_sweep<R, VT>(const BatchTab&, hipStream_t);        \
  template void launch_batch_iter_finalize<R, VT>(const BatchTab&, hipStream_t);     \
  template void launch_batch_iter_rescale<R, VT>(const BatchTab&, hipStream_t);      \
  template int sweep_batch_resident_blocks<R, VT>();                                 \
  template int sweep_resident_blocks<R, VT>();                                       \
  template int tile_resident_blocks<R, VT>();                                        \
  template int tile_batch_resident_blocks<R, VT>();                                  \
  template void launch_devices<R, VT>(const KArgs<R, VT>&, hipStream_t);            \
  template void launch_sweep<R, VT>(const KArgs<R, VT>&, hipStream_t);              \
  template void launch_finalize<R, VT>(const KArgs<R, VT>&, hipStream_t);           \
  template void launch_rescale<R, VT>(const KArgs<R, VT>&, hipStream_t);            \
  template void launch_export<R, VT>(const KArgs<R, VT>&, int, double*, hipStream_t);

OPF_INSTANTIATE(double, double)
OPF_INSTANTIATE(float, float)
OPF_INSTANTIATE(float, bf16_t)
template void launch_widen<float>(const KArgs<float, float>&, const KArgs<double, double>&, hipStream_t);
template void launch_widen<bf16_t>(const KArgs<float, bf16_t>&, const KArgs<double, double>&, hipStream_t);

}  // namespace opf
