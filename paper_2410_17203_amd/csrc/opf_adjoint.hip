// Reverse mode of unrolled message-passing iterations (arXiv 2410.17203,
// Section 4.4; the sensitivities of Section 5.5): derivatives of the final
// device powers and of the cost with respect to problem data, through the
// iterations, written by hand instead of recorded by a tracing framework.  The forward pass records the
// penalty schedule and snapshots of the iterate; the reverse pass walks the
// iterations backwards, recomputing from each snapshot which clips were
// active and applying the transposed piecewise-linear maps:
//
//   k_adj_sweep    reverse of the node update, the node averages and the line
//                  prox (the from node of each line stores its adjoint, both
//                  end nodes accumulate their own side, fixed order, no
//                  atomics), and the capacity derivative; each node row first
//                  sums, over the node's devices, the adjoint of the
//                  contingency means of W and thetabar that the next
//                  iteration's device step read (for itself and for the far
//                  node of each line);
//   k_adj_devices  reverse of the device step: the phase-dual update, the
//                  generator clip (the generator-limit derivative), the loads
//                  (the load derivative), and the inner ADMM of ramp
//                  generators and batteries, reversed through its inner
//                  iterations with the clip masks the recorded forward run
//                  kept (each tridiagonal solve is symmetric, so its
//                  transpose is the same solve).
//
// Notation of the forward (per contingency k, period t, line l with from node
// f and to node h): half = P / (2s) (outaged line: Td), theta1 = Tm + half,
// theta2 = Tm - half, v1 = sv (V1 + theta1 - TB_f), z1 = -P - W_f,
// z2 = P - W_h, xi1 = TB_f - v1, u = ca (z2 - z1) + cb (xi1 - xi2),
// P' = clip(u, -cap, cap), Tm' = (xi1 + xi2) / 2; node: pbar = sum / deg,
// U' = U + pbar, W' = U' + pbar, then W'' = W' + (su - 1) U', U'' = su U'.
#include <algorithm>

#include "opf_device.h"

namespace opf {

// Adjoint targets of one node row (16 bytes of contingencies): from the
// adjoint of (U'', W'', TB') and of the contingency means read by the next
// device step, the adjoints of the node's power and phase sums (divided by
// its degree) and of the incoming price U.
template <typename R, int VEC>
struct NodeAdj {
  R sp[VEC], sb[VEC], u_in[VEC];
};

// Adjoint of the contingency means of W and thetabar at node n, period t,
// that the next iteration's device step read: avgW enters each device's prox
// target with sign -1, avgTB its phase and phase-dual update (sums over the
// node's devices in CSR order).
template <typename R>
__device__ inline void dev_mean_adj(const AdjArgs<R>& a, int n, int t, R& sw, R& st) {
  const Topo& tp = a.tp;
  sw = R(0);
  st = R(0);
  for (int q = tp.node_nptr[n]; q < tp.node_nptr[n + 1]; ++q) {
    const int j = tp.node_nterm[q];
    sw -= a.dev_x[size_t(j) * tp.T + t];
    st += a.dev_t[size_t(j) * tp.T + t];
  }
}

// (mw, mt: dev_mean_adj of the node)
template <typename R, int VEC>
__device__ inline void node_adj(const AdjArgs<R>& a, size_t off, int n, R mw, R mt, int k0,
                                NodeAdj<R, VEC>& o) {
  using VR = Vec<R, VEC>;
  const Topo& tp = a.tp;
  const VR Ub = *reinterpret_cast<const VR*>(a.out.U + off);
  const VR Wb = *reinterpret_cast<const VR*>(a.out.W + off);
  const VR Tb = *reinterpret_cast<const VR*>(a.out.TB + off);
  const R iKp = R(1) / R(tp.Kp);
  const R aw = mw * iKp;
  const R at = mt * iKp;
  const R su = R(a.s.su_next);
  const R idg = R(tp.inv_deg[n]);
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const bool valid = k0 + e < tp.Kp;
    const R w2 = Wb.x[e] + aw;                       // adjoint of W''
    const R u1 = su * Ub.x[e] + (su - R(1)) * w2;    // adjoint of U'
    const R pb = u1 + R(2) * w2;                     // adjoint of pbar
    o.sp[e] = valid ? pb * idg : R(0);
    o.sb[e] = valid ? (Tb.x[e] + at) * idg : R(0);
    o.u_in[e] = valid ? u1 + w2 : R(0);
  }
}

// Reverse of one (period, node) row and one 16-byte vector of contingencies.
// GEN: the general line model (Section 2.3: DC links, per-contingency line
// parameters), whose special lines the forward took through line_prox_gen:
// per contingency a line is then an AC line with that contingency's
// susceptance and capacity (mode 0), out of service with its held half
// phase difference as state (mode 1: the N-1 outage, state Td, or a change
// that takes it out, state Tz), or a DC link (mode 2: flow at the clipped
// midpoint, half difference as state Hd).
template <typename R, bool GEN>
__device__ inline void adj_vec(const AdjArgs<R>& a, int row, int v, int q0, int q1, R mw, R mt,
                               R& gsp, R& gsb) {
  constexpr int VEC = 16 / sizeof(R);
  using VR = Vec<R, VEC>;
  using VI = Vec<int32_t, VEC>;
  const Topo& tp = a.tp;
  const int t = row / tp.N, n = row - t * tp.N;
  const int k0 = v * VEC;
  const size_t off = ck_off(t, n, k0, tp.N, tp.Kpp);
  const VI ok = *reinterpret_cast<const VI*>(tp.outage_k + k0);
  const VR Wo = *reinterpret_cast<const VR*>(a.A.W + off);
  const VR Bo = *reinterpret_cast<const VR*>(a.A.TB + off);
  const R* td_old = a.A.Td + size_t(t) * tp.Kpp + k0;
  const R* tdb_out = a.out.Td + size_t(t) * tp.Kpp + k0;
  R* tdb_in = a.in.Td + size_t(t) * tp.Kpp + k0;
  const R rp = R(a.s.rp), rt = R(a.s.rt), sv = R(a.s.sv);
  NodeAdj<R, VEC> me;
  node_adj<R, VEC>(a, off, n, mw, mt, k0, me);
  R accW[VEC], accB[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) accW[e] = accB[e] = R(0);
  for (int q = q0; q < q1; ++q) {
    const int2 term = tp.node_lterm[q];
    const int l = term.x >> 1, m = term.y;
    const bool to_end = term.x & 1;  // this node is the line's terminal-2 node
    const size_t ol = ck_off(t, l, k0, tp.L, tp.Kpp);
    const size_t oo = ck_off(t, m, k0, tp.N, tp.Kpp);
    const VR P = *reinterpret_cast<const VR*>(a.A.P + ol);
    const VR Tm = *reinterpret_cast<const VR*>(a.A.Tm + ol);
    const VR V1 = *reinterpret_cast<const VR*>(a.A.V1 + ol);
    const VR V2 = *reinterpret_cast<const VR*>(a.A.V2 + ol);
    const VR Wx = *reinterpret_cast<const VR*>(a.A.W + oo);
    const VR Bx = *reinterpret_cast<const VR*>(a.A.TB + oo);
    const R inv2s = R(tp.hinv_sus[l]), cap = R(tp.cap[l]);
    LineOut<R, VEC> o;
    bool special = false;
    int dci = -1;
    size_t oh = 0;
    if constexpr (GEN) {
      dci = tp.line_dc[l];
      special = dci >= 0 || tp.chg_ptr[l] != tp.chg_ptr[l + 1];
    }
    if (special) {
      VR Hx{};
      if (dci >= 0) {
        oh = ck_off(t, dci, k0, tp.Ldc, tp.Kpp);
        Hx = *reinterpret_cast<const VR*>(a.A.Hd + oh);
      }
      line_prox_gen<R, R, VEC>(tp, l, k0, ok, dci, Hx, td_old, a.A.Tz + size_t(t) * tp.Zc,
                               nullptr, P, Tm, V1, V2, to_end ? Wx : Wo, to_end ? Wo : Wx,
                               to_end ? Bx : Bo, to_end ? Bo : Bx, tp.Kp, rp, rt, sv, o);
    } else {
      line_prox<R, R, VEC>(P, Tm, V1, V2, to_end ? Wx : Wo, to_end ? Wo : Wx, to_end ? Bx : Bo,
                           to_end ? Bo : Bx, ok, l, td_old, k0, tp.Kp, inv2s, cap, rp, rt, sv, o);
    }
    NodeAdj<R, VEC> far;
    R fw, ft;
    dev_mean_adj<R>(a, m, t, fw, ft);
    node_adj<R, VEC>(a, oo, m, fw, ft, k0, far);
    const VR Pb = *reinterpret_cast<const VR*>(a.out.P + ol);
    const VR Tmb = *reinterpret_cast<const VR*>(a.out.Tm + ol);
    const VR V1b = *reinterpret_cast<const VR*>(a.out.V1 + ol);
    const VR V2b = *reinterpret_cast<const VR*>(a.out.V2 + ol);
    const R iden = R(1) / (R(2) * rp + R(2) * rt * inv2s * inv2s);
    const R ca0 = rp * iden, cb0 = rt * inv2s * iden;
    VR Pi, Ti, V1i, V2i;
    double* gc = a.gcap + ol;
    const R* tzb_out = GEN ? a.out.Tz + size_t(t) * tp.Zc : nullptr;
    R* tzb_in = GEN ? a.in.Tz + size_t(t) * tp.Zc : nullptr;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const bool valid = k0 + e < tp.Kp;
      const bool outg = ok.x[e] == l;
      // this contingency's line model, as line_prox_gen formed it
      int mode = outg ? 1 : 0, z = -1;
      R is2 = inv2s, cp = cap, ca = ca0, cb = cb0;
      bool cap_base = true;  // the capacity is the line's own (not a change's)
      if (GEN && special) {
        const int k = k0 + e;
        R sus = R(tp.sus[l]);
        cp = R(tp.cap[l]);
        mode = outg ? 1 : (dci >= 0 ? 2 : 0);
        for (int c = tp.chg_ptr[l]; c < tp.chg_ptr[l + 1]; ++c) {
          const LineChg ch = tp.chg[c];
          if (ch.k > k) break;
          if (ch.k != k) continue;
          cap_base = false;
          if (dci >= 0) {
            cp = R(ch.cap);
          } else if (ch.z >= 0) {
            mode = 1;
            z = ch.z;
          } else {
            sus = R(ch.sus);
            cp = R(ch.cap);
          }
        }
        is2 = R(0.5) / (mode == 0 ? sus : R(1));
        const R id = R(1) / (R(2) * rp + R(2) * rt * is2 * is2);
        ca = rp * id;
        cb = rt * is2 * id;
      }
      const R spf = to_end ? far.sp[e] : me.sp[e], sph = to_end ? me.sp[e] : far.sp[e];
      const R sbf = to_end ? far.sb[e] : me.sb[e], sbh = to_end ? me.sb[e] : far.sb[e];
      // adjoints of the line's outputs, including what the node sums took
      // and what the next iteration read of the held half difference
      R pt = Pb.x[e] + sph - spf;
      const R tt = Tmb.x[e] + sbf + sbh;
      R hb = sbf - sbh;
      // where the line holds its half phase difference (modes 1 and 2): Hd
      // for a DC link (outaged or not), Tz for a line a change takes out, Td
      // for the N-1 outage of an AC line; the next iteration read it there
      const int src = (GEN && dci >= 0) ? 2 : (mode == 1 ? (z >= 0 ? 3 : 1) : 0);
      if (src == 1) hb += tdb_out[e];
      if (GEN && src == 2) hb += a.out.Hd[oh + e];
      if (GEN && src == 3) hb += tzb_out[z];
      R x1, x2, z1b, z2b;
      if (mode == 1) {
        x1 = R(0.5) * (hb + tt);
        x2 = R(0.5) * (tt - hb);
        z1b = z2b = R(0);
      } else if (mode == 2) {  // DC link: u = (z2 - z1) / 2, half = (xi1 - xi2) / 2
        const bool pass = clip_pass(o.u[e], -cp, cp);
        const R ub = pass ? pt : R(0);
        if (!to_end && valid && !pass && cap_base) gc[e] += double(o.u[e] > cp ? pt : -pt);
        z2b = R(0.5) * ub;
        z1b = -z2b;
        x1 = R(0.5) * (hb + tt);
        x2 = R(0.5) * (tt - hb);
      } else {
        pt += hb * is2;
        const bool pass = clip_pass(o.u[e], -cp, cp);
        const R ub = pass ? pt : R(0);
        if (!to_end && valid && !pass && cap_base) gc[e] += double(o.u[e] > cp ? pt : -pt);
        z2b = ca * ub;
        z1b = -z2b;
        x1 = cb * ub + R(0.5) * tt;
        x2 = R(0.5) * tt - cb * ub;
      }
      const R v1b = V1b.x[e] - x1, v2b = V2b.x[e] - x2;
      const R th1b = sv * v1b, th2b = sv * v2b;
      const R hin = th1b - th2b;
      R pin = z2b - z1b;
      if (mode == 0) pin += hin * is2;
      Pi.x[e] = valid ? pin : R(0);
      Ti.x[e] = valid ? th1b + th2b : R(0);
      V1i.x[e] = valid ? sv * v1b : R(0);
      V2i.x[e] = valid ? sv * v2b : R(0);
      if (valid) {
        accW[e] += to_end ? -z2b : -z1b;
        accB[e] += to_end ? x2 - th2b : x1 - th1b;
      }
      if (!to_end && valid) {  // the held half difference the line read
        if (src == 1) tdb_in[e] = hin;
        if (GEN && src == 3) tzb_in[z] = hin;
        if (GEN && src == 2) {
          a.in.Hd[oh + e] = hin;
          if (outg) tdb_in[e] = R(0);  // (written by the forward, read by no line)
        }
      }
    }
    if (!to_end) {  // the from node stores the line's adjoint
      *reinterpret_cast<VR*>(a.in.P + ol) = Pi;
      *reinterpret_cast<VR*>(a.in.Tm + ol) = Ti;
      *reinterpret_cast<VR*>(a.in.V1 + ol) = V1i;
      *reinterpret_cast<VR*>(a.in.V2 + ol) = V2i;
    }
  }
  VR Ui, Wi, Bi;
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    Ui.x[e] = me.u_in[e];
    Wi.x[e] = accW[e];
    Bi.x[e] = accB[e];
    gsp += me.sp[e];
    gsb += me.sb[e];
  }
  *reinterpret_cast<VR*>(a.in.U + off) = Ui;
  *reinterpret_cast<VR*>(a.in.W + off) = Wi;
  *reinterpret_cast<VR*>(a.in.TB + off) = Bi;
}

template <typename R, bool GEN>
__global__ void __launch_bounds__(kBlock) k_adj_sweep(AdjArgs<R> a) {
  const int lpr = a.lanes_per_row, nv = a.nv;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int rw = lane / lpr, q = lane - rw * lpr;
  const int rows_per_wave = kWave / lpr;
  const int64_t NT = int64_t(a.tp.N) * a.tp.T;
  for (int64_t gi = blockIdx.x; gi < a.n_grps; gi += gridDim.x) {
    const int64_t row = (gi * (kBlock / kWave) + w) * rows_per_wave + rw;
    const bool act = row < NT;
    R gsp = R(0), gsb = R(0);
    int n = 0, t = 0;
    if (act) {
      t = int(row / a.tp.N);
      n = int(row - int64_t(t) * a.tp.N);
      const int q0 = a.tp.node_lptr[n], q1 = a.tp.node_lptr[n + 1];
      R mw, mt;
      dev_mean_adj<R>(a, n, t, mw, mt);
      for (int v = q; v < nv; v += lpr) adj_vec<R, GEN>(a, int(row), v, q0, q1, mw, mt, gsp, gsb);
    }
    for (int d = lpr >> 1; d > 0; d >>= 1) {
      gsp += __shfl_xor(gsp, d);
      gsb += __shfl_xor(gsb, d);
    }
    if (act && q == 0) {
      a.gsp[size_t(n) * a.tp.T + t] = gsp;
      a.gsb[size_t(n) * a.tp.T + t] = gsb;
    }
  }
}

// Reverse of the ramp generator's inner ADMM: walks the inner iterations
// backwards with the clip masks the recorded forward run kept (masks: this
// iteration's).  pb: adjoint of the output power; adj: adjoint of the inner
// state after the call (read) and before it (written back, lambdas times
// su).  Returns the adjoint of the prox target X.
template <typename R, int E>
__device__ void ramp_adj(const Topo& tp, const uint32_t* masks, R* adj, int r, int g, R rho_hat,
                         R omega, R su, int n_inner, int lane, const R (&pb)[E], R (&Xb)[E],
                         double* gpmax) {
  const int T = tp.T;
  const size_t nRT = size_t(tp.nR) * T;
  const size_t o = size_t(r) * T;
  ClipMasks<E, 2> mk;
  masks_load<E, 2>(masks + mask_ramp_off(r, E), mk, lane);
  const R c2 = R(tp.gen_c2[g]);
  const R w = R(2) * c2 + rho_hat;
  const R eo = -omega;
  R mul[E], invm[E];
  thomas_factors<R, E>(T, eo, [&](int t) { return w + omega + omega * R((t > 0) + (t < T - 1)); },
                       lane, mul, invm);
  R Bb[E], Lb[E], Br[E], Lr[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    Bb[e] = t < T ? adj[0 * nRT + o + t] : R(0);
    Lb[e] = t < T ? adj[1 * nRT + o + t] : R(0);
    Br[e] = t < T - 1 ? adj[2 * nRT + o + t] : R(0);
    Lr[e] = t < T - 1 ? adj[3 * nRT + o + t] : R(0);
    Xb[e] = R(0);
  }
  for (int it = n_inner - 1; it >= 0; --it) {
    R xb[E], dpb[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      xb[e] = (it == n_inner - 1 && t < T) ? pb[e] : R(0);
      dpb[e] = R(0);
      if (t < T) {
        const R bn = Bb[e] - Lb[e];
        const R thru = mk.pass(0, it, e) ? bn : R(0);
        if (mk.at_high(0, it, e)) gpmax[size_t(g) * T + t] += double(bn);
        xb[e] += Lb[e] + thru;
        Lb[e] += thru;
      }
      if (t < T - 1) {
        const R rn = Br[e] - Lr[e];
        const R thru = mk.pass(1, it, e) ? rn : R(0);
        dpb[e] = Lr[e] + thru;
        Lr[e] += thru;
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const R prev = prev_slot<R, E>(dpb, e);  // dp_{t-1} = x_t - x_{t-1}
      xb[e] += prev - dpb[e];
    }
    thomas_solve<R, E>(T, eo, mul, invm, xb, lane);  // symmetric: transpose solve
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      const R nx = next_slot<R, E>(xb, e);
      if (t < T) {
        Xb[e] += rho_hat * xb[e];
        Bb[e] = omega * xb[e];
        Lb[e] -= omega * xb[e];
      }
      if (t < T - 1) {
        const R qb = omega * (nx - xb[e]);
        Br[e] = qb;
        Lr[e] -= qb;
      } else {
        Br[e] = Lr[e] = R(0);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    if (t < T) {
      adj[0 * nRT + o + t] = Bb[e];
      adj[1 * nRT + o + t] = su * Lb[e];
      adj[2 * nRT + o + t] = Br[e];
      adj[3 * nRT + o + t] = su * Lr[e];
    }
  }
}

// Reverse of the battery's inner ADMM; db: adjoint of the discharge delta of
// the last x-update (the objective's alpha * sum delta), besides pb.
template <typename R, int E>
__device__ void battery_adj(const Topo& tp, const uint32_t* masks, R* adj, int b, R rho_hat,
                            R omega, R su, int n_inner, int lane, const R (&pb)[E], R db,
                            R (&Xb)[E]) {
  const int T = tp.T;
  const size_t nBT = size_t(tp.B) * T;
  const size_t o = size_t(b) * T;
  ClipMasks<E, 3> mk;
  masks_load<E, 3>(masks + mask_bat_off(tp.nR, b, E), mk, lane);
  const BatK<R> k(tp, b, rho_hat, omega);
  const R eo = -k.iw;
  R mul[E], invm[E];
  thomas_factors<R, E>(T, eo, [&](int t) { return k.kappa + k.iw * R((t < T - 1) + (t > 0)); },
                       lane, mul, invm);
  R Bc[E], Lc[E], Bd[E], Ld[E], Bs[E], Ls[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    const bool ok = t < T, oks = t >= 1 && t < T;
    Bc[e] = ok ? adj[0 * nBT + o + t] : R(0);
    Lc[e] = ok ? adj[1 * nBT + o + t] : R(0);
    Bd[e] = ok ? adj[2 * nBT + o + t] : R(0);
    Ld[e] = ok ? adj[3 * nBT + o + t] : R(0);
    Bs[e] = oks ? adj[4 * nBT + o + t] : R(0);
    Ls[e] = oks ? adj[5 * nBT + o + t] : R(0);
    Xb[e] = R(0);
  }
  for (int it = n_inner - 1; it >= 0; --it) {
    R cb[E], dlb[E], sb[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      const bool lastit = it == n_inner - 1;
      cb[e] = dlb[e] = sb[e] = R(0);
      if (t < T) {
        cb[e] = lastit ? -pb[e] : R(0);
        dlb[e] = lastit ? pb[e] + db : R(0);
        R bn = Bc[e] - Lc[e];
        R thru = mk.pass(0, it, e) ? bn : R(0);
        cb[e] += Lc[e] + thru;
        Lc[e] += thru;
        bn = Bd[e] - Ld[e];
        thru = mk.pass(1, it, e) ? bn : R(0);
        dlb[e] += Ld[e] + thru;
        Ld[e] += thru;
      }
      if (t >= 1 && t < T) {
        const R bn = Bs[e] - Ls[e];
        const R thru = mk.pass(2, it, e) ? bn : R(0);
        sb[e] = Ls[e] + thru;
        Ls[e] += thru;
      }
    }
    // nu_t enters c_t, delta_t, s_t (+1/omega) and s_{t+1} (-1/omega)
    R nub[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      const R sn = next_slot<R, E>(sb, e);
      nub[e] = t < T ? k.hgc * cb[e] + k.hgd * dlb[e] + (sb[e] - sn) * k.iw : R(0);
    }
    thomas_solve<R, E>(T, eo, mul, invm, nub, lane);  // symmetric: transpose solve
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      const R rprev = prev_slot<R, E>(nub, e);  // rhs_{t-1} holds + qs_t
      if (t < T) {
        const R qsb = sb[e] + (t >= 1 ? rprev : R(0)) - nub[e];
        const R hrcb = cb[e] - k.eta * nub[e];
        const R hrdb = dlb[e] + nub[e];
        const R rcb = k.h11 * hrcb + k.h12 * hrdb;
        const R rdb = k.h12 * hrcb + k.h11 * hrdb;
        Bc[e] = omega * rcb;
        Lc[e] -= omega * rcb;
        Bd[e] = omega * rdb;
        Ld[e] -= omega * rdb;
        Xb[e] += rho_hat * (rdb - rcb);
        if (t >= 1) {
          Bs[e] = qsb;
          Ls[e] -= qsb;
        } else {
          Bs[e] = Ls[e] = R(0);
        }
      } else {
        Bc[e] = Lc[e] = Bd[e] = Ld[e] = Bs[e] = Ls[e] = R(0);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    if (t < T) {
      adj[0 * nBT + o + t] = Bc[e];
      adj[1 * nBT + o + t] = su * Lc[e];
      adj[2 * nBT + o + t] = Bd[e];
      adj[3 * nBT + o + t] = su * Ld[e];
      if (t >= 1) {
        adj[4 * nBT + o + t] = Bs[e];
        adj[5 * nBT + o + t] = su * Ls[e];
      }
    }
  }
}

// Reverse of the device step, one device per wavefront (T across lanes).
template <typename R, int E>
__global__ void __launch_bounds__(kBlock) k_adj_devices(AdjArgs<R> a) {
  const Topo& tp = a.tp;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * (kBlock / kWave) + w;
  if (j >= tp.Jnc) return;
  const int T = tp.T;
  const int n = tp.nc_node[j];
  const R sv = R(a.s.sv), su = R(a.s.su);
  const R rho_hat = R(tp.Kp) * R(a.s.rp);
  const R omega = R(a.omega_scale) * rho_hat;
  R X[E], pb[E], Xb[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    X[e] = pb[e] = Xb[e] = R(0);
    if (t < T) {
      const size_t o = size_t(j) * T + t, on = size_t(n) * T + t;
      pb[e] = a.dev_p[o] + a.gsp[on];
      const R thb = a.dev_th[o] + a.gsb[on];
      const R vtot = a.dev_v[o] - thb;  // adjoint of the updated phase dual
      a.dev_t[o] = thb - sv * vtot;
      a.dev_v[o] = sv * vtot;
      a.dev_th[o] = sv * vtot;
      X[e] = a.pnc[o] - a.avgW[on];
    }
  }
  if (j < tp.G) {
    const int r = tp.ramp_idx[j];
    if (r < 0) {
      const R c2 = R(tp.gen_c2[j]), c1 = R(tp.gen_c1[j]);
      const R slope = rho_hat / (R(2) * c2 + rho_hat);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int t = lane * E + e;
        if (t < T) {
          const R y = gen_target(X[e], c1, c2, rho_hat);
          const bool pass = clip_pass(y, R(tp.gen_pmin[size_t(j) * T + t]),
                                      R(tp.gen_pmax[size_t(j) * T + t]));
          Xb[e] = pass ? slope * pb[e] : R(0);
          if (y > R(tp.gen_pmax[size_t(j) * T + t])) a.gpmax[size_t(j) * T + t] += double(pb[e]);
        }
      }
    } else {
      ramp_adj<R, E>(tp, a.masks, a.ramp_adj, r, j, rho_hat, omega, su, a.inner_iters, lane, pb,
                     Xb, a.gpmax);
    }
  } else if (j < tp.G + tp.D) {
    const int d = j - tp.G;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      if (t < T) a.gload[size_t(d) * T + t] -= double(pb[e]);  // p = -d
    }
  } else {
    const int b = j - tp.G - tp.D;
    const R db = a.s.last ? R(a.w_obj * tp.bat_alpha[b]) : R(0);
    battery_adj<R, E>(tp, a.masks, a.bat_adj, b, rho_hat, omega, su, a.inner_iters, lane, pb, db,
                      Xb);
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    if (t < T) {
      const size_t o = size_t(j) * T + t;
      a.dev_p[o] = Xb[e];  // the prox target is p - avgW
      a.dev_x[o] = Xb[e];
    }
  }
}

// Cotangent of the final iterate: the caller's weights on the device powers
// plus w_obj times the derivative of the generator cost.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_adj_init(AdjArgs<R> a, const double* cot) {
  const Topo& tp = a.tp;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= int64_t(tp.Jnc) * tp.T) return;
  const int j = int(i / tp.T);
  double v = cot ? cot[i] : 0.0;
  if (j < tp.G) v += a.w_obj * (2.0 * tp.gen_c2[j] * double(a.pnc[i]) + tp.gen_c1[j]);
  a.dev_p[i] = R(v);
}

// Capacity derivative: sum over periods and contingencies.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_adj_cap(AdjArgs<R> a, double* grad) {
  const Topo& tp = a.tp;
  const int l = blockIdx.x;
  __shared__ double sh[kBlock / kWave];
  double s = 0.0;
  const int64_t per = int64_t(tp.T) * tp.Kpp;
  for (int64_t i = threadIdx.x; i < per; i += kBlock) {
    const int t = int(i / tp.Kpp), k = int(i - int64_t(t) * tp.Kpp);
    s += a.gcap[ck_off(t, l, k, tp.L, tp.Kpp)];
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) grad[l] = s;
}

__global__ void __launch_bounds__(kBlock) k_copy(CopyList cl) {
  const int i = blockIdx.y;
  const char* src = cl.src[i];
  char* dst = cl.dst[i];
  const size_t nb = cl.bytes[i];
  const size_t n16 = nb / 16;
  const size_t stride = size_t(gridDim.x) * kBlock;
  for (size_t q = size_t(blockIdx.x) * kBlock + threadIdx.x; q < n16; q += stride)
    reinterpret_cast<uint4*>(dst)[q] = reinterpret_cast<const uint4*>(src)[q];
  for (size_t q = n16 * 16 + size_t(blockIdx.x) * kBlock + threadIdx.x; q < nb; q += stride)
    dst[q] = src[q];
}

// ---------------------------------------------------------------------------
// Launchers.

template <typename R>
void launch_adj_iteration(const AdjArgs<R>& a, hipStream_t s) {
  const int64_t grid = std::min<int64_t>(a.n_grps, 8192);
  if (a.tp.Ldc > 0 || a.tp.n_chg > 0)
    k_adj_sweep<R, true><<<int(grid), kBlock, 0, s>>>(a);
  else
    k_adj_sweep<R, false><<<int(grid), kBlock, 0, s>>>(a);
  const int nblk = (a.tp.Jnc + 3) / 4;
  if (nblk == 0) return;
  const int E = (a.tp.T + kWave - 1) / kWave;
  switch (E) {
    case 1: k_adj_devices<R, 1><<<nblk, kBlock, 0, s>>>(a); break;
    case 2: k_adj_devices<R, 2><<<nblk, kBlock, 0, s>>>(a); break;
    case 3: k_adj_devices<R, 3><<<nblk, kBlock, 0, s>>>(a); break;
    default: k_adj_devices<R, 4><<<nblk, kBlock, 0, s>>>(a); break;
  }
}

template <typename R>
void launch_adj_init(const AdjArgs<R>& a, const double* cot, hipStream_t s) {
  const int64_t n = int64_t(a.tp.Jnc) * a.tp.T;
  if (n == 0) return;
  k_adj_init<R><<<int((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(a, cot);
}

template <typename R>
void launch_adj_cap(const AdjArgs<R>& a, double* grad, hipStream_t s) {
  if (a.tp.L == 0) return;
  k_adj_cap<R><<<a.tp.L, kBlock, 0, s>>>(a, grad);
}

void launch_copy(const CopyList& cl, hipStream_t s) {
  if (cl.n == 0) return;
  size_t mx = 0;
  for (int i = 0; i < cl.n; ++i) mx = std::max(mx, cl.bytes[i]);
  const size_t blocks = std::min<size_t>(1024, (mx / 16 + kBlock - 1) / kBlock + 1);
  k_copy<<<dim3(unsigned(blocks), unsigned(cl.n)), kBlock, 0, s>>>(cl);
}

template void launch_adj_iteration<double>(const AdjArgs<double>&, hipStream_t);
template void launch_adj_iteration<float>(const AdjArgs<float>&, hipStream_t);
template void launch_adj_init<double>(const AdjArgs<double>&, const double*, hipStream_t);
template void launch_adj_init<float>(const AdjArgs<float>&, const double*, hipStream_t);
template void launch_adj_cap<double>(const AdjArgs<double>&, double*, hipStream_t);
template void launch_adj_cap<float>(const AdjArgs<float>&, double*, hipStream_t);

}  // namespace opf
