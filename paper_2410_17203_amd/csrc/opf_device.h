// Device helpers shared by the forward kernels (opf_kernels.hip) and the
// adjoint kernels (opf_adjoint.hip): vector types and streaming loads, the
// XCD-aware work split, deterministic reductions, wavefront linear
// recurrences and tridiagonal solves, and the proximal operators whose exact
// arithmetic the adjoint must replay (line prox, Section 4.2; the inner ADMM
// of the ramp generator and the battery, Appendix D).
#pragma once

#include "opf_internal.h"


// 1: rows read once per sweep (own price row) and all rows written by it use
// non-temporal loads and stores, so they do not evict from L2 the line and
// node rows that neighbouring nodes read again shortly after.
#ifndef OPF_NT
#define OPF_NT 1
#endif
// Line terminals of a node taken per step of the single-instance node-row
// sweep (1 or 2): all loads of a step are issued before any of them is used.
#ifndef OPF_SWEEP_BATCH
#define OPF_SWEEP_BATCH 1
#endif
// Minimum waves per SIMD requested for the sweep (0: compiler's choice); a
// higher value caps its registers so that more waves hide memory latency.
#ifndef OPF_SWEEP_WAVES
#define OPF_SWEEP_WAVES 0
#endif
#if OPF_SWEEP_WAVES > 0
#define OPF_SWEEP_ATTR __attribute__((amdgpu_waves_per_eu(OPF_SWEEP_WAVES)))
#else
#define OPF_SWEEP_ATTR
#endif


namespace opf {


template <typename T, int N>
struct alignas(sizeof(T) * N) Vec {
  T x[N];
};

// Storage conversion of the phase duals (FP32 arithmetic on BF16 storage).
template <typename VT, typename R>
struct DIO;
template <typename R>
struct DIO<R, R> {
  __device__ static R in(R v) { return v; }
  __device__ static R out(R v) { return v; }
};
template <>
struct DIO<bf16_t, float> {
  __device__ static float in(bf16_t v) { return __uint_as_float(uint32_t(v.u) << 16); }
  __device__ static bf16_t out(float f) {
    uint32_t u = __float_as_uint(f);
    bf16_t r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      r.u = uint16_t((u >> 16) | 0x40u);
      return r;
    }
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    r.u = uint16_t(u >> 16);
    return r;
  }
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// 16- or 8-byte vector load/store that bypasses L2 retention when OPF_NT.
template <typename V>
__device__ inline V ld_stream(const V* p) {
  static_assert(sizeof(V) == 16 || sizeof(V) == 8, "vector size");
#if OPF_NT
  if constexpr (sizeof(V) == 16) {
    return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p)));
  } else {
    return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p)));
  }
#else
  return *p;
#endif
}
template <typename V>
__device__ inline void st_stream(V* p, const V& v) {
  static_assert(sizeof(V) == 16 || sizeof(V) == 8, "vector size");
#if OPF_NT
  if constexpr (sizeof(V) == 16) {
    __builtin_nontemporal_store(__builtin_bit_cast(u32x4, v), reinterpret_cast<u32x4*>(p));
  } else {
    __builtin_nontemporal_store(__builtin_bit_cast(u32x2, v), reinterpret_cast<u32x2*>(p));
  }
#else
  *p = v;
#endif
}

// x / d for a small positive integer d from r = 1/d (correctly rounded):
// one residual correction of x * r, which rounds like the division except in
// rare ties, at three instructions instead of a full IEEE division.
template <typename R>
__device__ inline R div_by(R x, R d, R r) {
  const R q = x * r;
  return fma(fma(-q, d, x), r, q);
}

template <typename R>
__device__ inline R clampv(R x, R lo, R hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

// Workgroups are dealt to the 8 XCDs round-robin by id.  Work items [0, n)
// are split into 8 contiguous ranges, one per XCD, and the nb/8 blocks of an
// XCD sweep their range together as one moving front (block j of the XCD
// takes items j, j + nb/8, ...), so the line and node rows that neighbouring
// items share are reused from that XCD's L2 shortly after first use.  nb must
// be a multiple of 8.
struct Sweep {
  int64_t first, end;
  int step;
};
#ifndef OPF_XCD_SWEEP
#define OPF_XCD_SWEEP 1
#endif
__device__ inline Sweep xcd_sweep(int b, int nb, int64_t n) {
  Sweep s;
#if OPF_XCD_SWEEP
  const int x = b & 7, j = b >> 3, per = nb >> 3;
  s.first = n * x / 8 + j;
  s.end = n * (x + 1) / 8;
  s.step = per;
#else
  s.first = b;
  s.end = n;
  s.step = nb;
#endif
  return s;
}

// Waits until this wave's LDS operations have completed (lgkmcnt(0); the
// vector-memory and export counters are left alone; gfx9 encoding).
__device__ inline void lds_wait() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (a full __syncthreads also waits for every
// outstanding global load and store of the wave).  For phases that exchange
// data through LDS and never read back global memory written by the
// workgroup.  The wave's own LDS writes are waited for explicitly before
// the barrier: the workgroup-scope fence alone let the compiler drop that
// wait on a loop back-edge, and another wave then read stale LDS after the
// barrier.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  lds_wait();
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ inline double wave_sum(double v) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

// Deterministic block sum over NT threads; the result is valid in thread 0.
template <int NT = kBlock>
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  lds_wait();
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / kWave; ++i) r += sh[i];
  lds_wait();
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Wavefront linear recurrences.  Element t of a length-T sequence lives in
// lane t / E, slot t % E.  fwd: x_t = a_t x_{t-1} + b_t with x_{-1} = 0;
// bwd: x_t = a_t x_{t+1} + b_t with x_T = 0.  Padding slots must hold the
// identity map (a = 1, b = 0).  The result overwrites b.

template <typename R, int E>
__device__ inline void scan_fwd(const R (&a)[E], R (&b)[E], int lane) {
  R A = R(1), B = R(0);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    B = a[e] * B + b[e];
    A = a[e] * A;
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const R pA = __shfl_up(A, d);
    const R pB = __shfl_up(B, d);
    if (lane >= d) {
      B = A * pB + B;
      A = A * pA;
    }
  }
  R x = __shfl_up(B, 1);
  if (lane == 0) x = R(0);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    x = a[e] * x + b[e];
    b[e] = x;
  }
}

template <typename R, int E>
__device__ inline void scan_bwd(const R (&a)[E], R (&b)[E], int lane) {
  R A = R(1), B = R(0);
#pragma unroll
  for (int e = E - 1; e >= 0; --e) {
    B = a[e] * B + b[e];
    A = a[e] * A;
  }
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const R pA = __shfl_down(A, d);
    const R pB = __shfl_down(B, d);
    if (lane + d < kWave) {
      B = A * pB + B;
      A = A * pA;
    }
  }
  R x = __shfl_down(B, 1);
  if (lane == kWave - 1) x = R(0);
#pragma unroll
  for (int e = E - 1; e >= 0; --e) {
    x = a[e] * x + b[e];
    b[e] = x;
  }
}

// Thomas factors of a tridiagonal matrix with diagonal diag(t) and constant
// off-diagonal eo: mul_t = eo / m_{t-1}, inv_m_t = 1 / m_t for this lane's
// slots (each lane runs the pivot recurrence up to its last slot).
template <typename R, int E, typename Diag>
__device__ inline void thomas_factors(int T, R eo, Diag diag, int lane, R (&mul)[E], R (&invm)[E]) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    mul[e] = R(0);
    invm[e] = R(0);
  }
  const int t0 = lane * E;
  const int tend = min(T, t0 + E);
  R mprev = R(1);
  for (int t = 0; t < tend; ++t) {
    const R mu = (t == 0) ? R(0) : eo / mprev;
    const R m = diag(t) - mu * eo;
    if (t >= t0) {
      mul[t - t0] = mu;
      invm[t - t0] = R(1) / m;
    }
    mprev = m;
  }
}

// Solves the tridiagonal system whose factors come from thomas_factors;
// rhs in x on entry, solution in x on exit.
template <typename R, int E>
__device__ inline void thomas_solve(int T, R eo, const R (&mul)[E], const R (&invm)[E],
                                    R (&x)[E], int lane) {
  R a[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool ok = lane * E + e < T;
    a[e] = ok ? -mul[e] : R(1);
    if (!ok) x[e] = R(0);
  }
  scan_fwd<R, E>(a, x, lane);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool ok = lane * E + e < T;
    a[e] = ok ? -eo * invm[e] : R(1);
    x[e] = ok ? invm[e] * x[e] : R(0);
  }
  scan_bwd<R, E>(a, x, lane);
}

// Value of slot e's predecessor (t - 1) and successor (t + 1) in the wave.
template <typename R, int E>
__device__ inline R prev_slot(const R (&v)[E], int e) {
  R up = __shfl_up(v[E - 1], 1);
  if ((threadIdx.x & 63) == 0) up = R(0);
  return e > 0 ? v[e > 0 ? e - 1 : 0] : up;
}
template <typename R, int E>
__device__ inline R next_slot(const R (&v)[E], int e) {
  R dn = __shfl_down(v[0], 1);
  if ((threadIdx.x & 63) == kWave - 1) dn = R(0);
  return e < E - 1 ? v[e < E - 1 ? e + 1 : 0] : dn;
}


// ---------------------------------------------------------------------------
// Step 2 for time-coupled devices: inner ADMM (Appendix D) with the device
// equalities in the x-update and the bounds split off (penalty omega).
//
// The forward pass keeps no record of which bounds were active; the adjoint
// replays the same code with a recorder that keeps two bits per (inner
// iteration, period, bound): the clip let its argument through
// (lo <= y <= hi, derivative 1), and the argument was above the upper bound
// (derivative 1 with respect to that bound).
struct NoMasks {
  __device__ void rec(int, int, int, bool, bool) {}
};
template <int E, int NB>
struct ClipMasks {
  uint32_t thru[NB][E];  // clip let its argument through
  uint32_t high[NB][E];  // clipped at the upper bound
  __device__ ClipMasks() {
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int e = 0; e < E; ++e) thru[b][e] = high[b][e] = 0u;
  }
  __device__ void rec(int bound, int it, int e, bool pass, bool hi) {
    if (pass) thru[bound][e] |= 1u << it;
    if (hi) high[bound][e] |= 1u << it;
  }
  __device__ bool pass(int bound, int it, int e) const { return (thru[bound][e] >> it) & 1u; }
  __device__ bool at_high(int bound, int it, int e) const { return (high[bound][e] >> it) & 1u; }
};

template <int E, int NB>
__device__ inline void masks_store(uint32_t* dst, const ClipMasks<E, NB>& m, int lane) {
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      dst[((b * 2 + 0) * E + e) * kWave + lane] = m.thru[b][e];
      dst[((b * 2 + 1) * E + e) * kWave + lane] = m.high[b][e];
    }
}

template <int E, int NB>
__device__ inline void masks_load(const uint32_t* src, ClipMasks<E, NB>& m, int lane) {
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      m.thru[b][e] = src[((b * 2 + 0) * E + e) * kWave + lane];
      m.high[b][e] = src[((b * 2 + 1) * E + e) * kWave + lane];
    }
}

template <typename R>
__device__ inline bool clip_pass(R y, R lo, R hi) {
  return !(y < lo) && !(y > hi);
}

// Ramp-limited generator: min c2|p|^2 + c1'p + rho_hat/2 |p - X|^2 over
// pmin <= p <= pmax, |p_{t+1} - p_t| <= Rl.  x-update matrix
// (2 c2 + rho_hat + omega) I + omega D'D, tridiagonal.  The inner state
// (beta_box, lambda_box, beta_ramp, lambda_ramp) is read from st_in (lambda
// scaled by su, the pending penalty ratio) and, if st_out is not null,
// written back there.  Bounds recorded: 0 = box, 1 = ramp.
template <typename R, int E, typename M>
__device__ void ramp_prox(const Topo& tp, const R* st_in, R* st_out, int r, int g, const R (&X)[E],
                          R rho_hat, R omega, R su, int n_inner, int lane, R (&p)[E], M& masks) {
  const int T = tp.T;
  const size_t nRT = size_t(tp.nR) * T;
  const size_t o = size_t(r) * T;
  const R c2 = R(tp.gen_c2[g]), c1 = R(tp.gen_c1[g]), Rl = R(tp.gen_ramp[g]);
  const R w = R(2) * c2 + rho_hat;
  R Bb[E], Lb[E], Br[E], Lr[E], lo[E], hi[E], base[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    if (t < T) {
      Bb[e] = st_in[0 * nRT + o + t];
      Lb[e] = su * st_in[1 * nRT + o + t];
      Br[e] = (t < T - 1) ? st_in[2 * nRT + o + t] : R(0);
      Lr[e] = (t < T - 1) ? su * st_in[3 * nRT + o + t] : R(0);
      lo[e] = R(tp.gen_pmin[size_t(g) * T + t]);
      hi[e] = R(tp.gen_pmax[size_t(g) * T + t]);
      base[e] = rho_hat * X[e] - c1;
    } else {
      Bb[e] = Lb[e] = Br[e] = Lr[e] = lo[e] = hi[e] = base[e] = R(0);
    }
  }
  const R eo = -omega;
  R mul[E], invm[E];
  thomas_factors<R, E>(T, eo, [&](int t) { return w + omega + omega * R((t > 0) + (t < T - 1)); },
                       lane, mul, invm);
  R x[E];
  for (int it = 0; it < n_inner; ++it) {
    R qr[E];
#pragma unroll
    for (int e = 0; e < E; ++e) qr[e] = Br[e] - Lr[e];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const R qprev = prev_slot<R, E>(qr, e);
      x[e] = base[e] + omega * ((Bb[e] - Lb[e]) + qprev - qr[e]);
    }
    thomas_solve<R, E>(T, eo, mul, invm, x, lane);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      const R xn = next_slot<R, E>(x, e);
      if (t < T) {
        const R y = x[e] + Lb[e];
        masks.rec(0, it, e, clip_pass(y, lo[e], hi[e]), y > hi[e]);
        const R bnew = clampv(y, lo[e], hi[e]);
        Lb[e] += x[e] - bnew;
        Bb[e] = bnew;
      }
      if (t < T - 1) {
        const R dp = xn - x[e];
        const R y = dp + Lr[e];
        masks.rec(1, it, e, clip_pass(y, -Rl, Rl), y > Rl);
        const R rnew = clampv(y, -Rl, Rl);
        Lr[e] += dp - rnew;
        Br[e] = rnew;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    p[e] = x[e];
    if (st_out != nullptr && t < T) {
      st_out[0 * nRT + o + t] = Bb[e];
      st_out[1 * nRT + o + t] = Lb[e];
      st_out[2 * nRT + o + t] = Br[e];
      st_out[3 * nRT + o + t] = Lr[e];
    }
  }
}

// Battery: min alpha 1'delta + rho_hat/2 |delta - c - X|^2 subject to
// s_{t+1} = s_t + eta c_t - delta_t, s_0 = s_T = 0, and bounds on c, delta,
// s_1..s_{T-1}.  Eliminating (c, delta) per period leaves a tridiagonal
// system in the dynamics multipliers nu.  Constants of the elimination:
template <typename R>
struct BatK {
  R Pc, smax, eta, alpha, h11, h12, hgc, hgd, kappa, iw;
  __device__ BatK(const Topo& tp, int b, R rho_hat, R omega) {
    Pc = R(tp.bat_P[b]);
    smax = R(tp.bat_dur[b]) * Pc;
    eta = R(tp.bat_eta[b]);
    alpha = R(tp.bat_alpha[b]);
    const R det = omega * (R(2) * rho_hat + omega);
    h11 = (rho_hat + omega) / det;
    h12 = rho_hat / det;
    hgc = h11 * eta - h12;  // H^-1 g, g = (eta, -1)
    hgd = h12 * eta - h11;
    kappa = eta * hgc - hgd;  // g' H^-1 g
    iw = R(1) / omega;
  }
};

// Inner state (beta/lambda of charge, discharge, state of charge) is read
// from st_in (lambdas scaled by su) and written to st_out if not null.
// Outputs the power delta - c of the last x-update and adds alpha * sum of
// delta to obj.  Bounds recorded: 0 = charge, 1 = discharge, 2 = state of
// charge.
template <typename R, int E, typename M>
__device__ void battery_prox(const Topo& tp, const R* st_in, R* st_out, int b, const R (&X)[E],
                             R rho_hat, R omega, R su, int n_inner, int lane, R (&p)[E],
                             double& obj, M& masks) {
  const int T = tp.T;
  const size_t nBT = size_t(tp.B) * T;
  const size_t o = size_t(b) * T;
  const BatK<R> k(tp, b, rho_hat, omega);
  R Bc[E], Lc[E], Bd[E], Ld[E], Bs[E], Ls[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    const bool ok = t < T, oks = t >= 1 && t < T;
    Bc[e] = ok ? st_in[0 * nBT + o + t] : R(0);
    Lc[e] = ok ? su * st_in[1 * nBT + o + t] : R(0);
    Bd[e] = ok ? st_in[2 * nBT + o + t] : R(0);
    Ld[e] = ok ? su * st_in[3 * nBT + o + t] : R(0);
    Bs[e] = oks ? st_in[4 * nBT + o + t] : R(0);
    Ls[e] = oks ? su * st_in[5 * nBT + o + t] : R(0);
  }
  R mul[E], invm[E];
  const R eo = -k.iw;
  thomas_factors<R, E>(T, eo, [&](int t) { return k.kappa + k.iw * R((t < T - 1) + (t > 0)); },
                       lane, mul, invm);
  R c[E], dl[E];
  for (int it = 0; it < n_inner; ++it) {
    R qs[E], nu[E], hrc[E], hrd[E];
#pragma unroll
    for (int e = 0; e < E; ++e) qs[e] = Bs[e] - Ls[e];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      const R rc = omega * (Bc[e] - Lc[e]) - rho_hat * X[e];
      const R rd = omega * (Bd[e] - Ld[e]) + rho_hat * X[e] - k.alpha;
      hrc[e] = k.h11 * rc + k.h12 * rd;
      hrd[e] = k.h12 * rc + k.h11 * rd;
      const R qn = next_slot<R, E>(qs, e);
      nu[e] = (t < T - 1 ? qn : R(0)) - qs[e] - (k.eta * hrc[e] - hrd[e]);
    }
    thomas_solve<R, E>(T, eo, mul, invm, nu, lane);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = lane * E + e;
      const R np = prev_slot<R, E>(nu, e);
      c[e] = hrc[e] + nu[e] * k.hgc;
      dl[e] = hrd[e] + nu[e] * k.hgd;
      if (t < T) {
        R y = c[e] + Lc[e];
        masks.rec(0, it, e, clip_pass(y, R(0), k.Pc), y > k.Pc);
        R nb = clampv(y, R(0), k.Pc);
        Lc[e] += c[e] - nb;
        Bc[e] = nb;
        y = dl[e] + Ld[e];
        masks.rec(1, it, e, clip_pass(y, R(0), k.Pc), y > k.Pc);
        nb = clampv(y, R(0), k.Pc);
        Ld[e] += dl[e] - nb;
        Bd[e] = nb;
      }
      if (t >= 1 && t < T) {
        const R s = qs[e] + (nu[e] - np) * k.iw;
        const R y = s + Ls[e];
        masks.rec(2, it, e, clip_pass(y, R(0), k.smax), y > k.smax);
        const R nb = clampv(y, R(0), k.smax);
        Ls[e] += s - nb;
        Bs[e] = nb;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = lane * E + e;
    p[e] = dl[e] - c[e];
    if (t < T) {
      obj += double(k.alpha) * double(dl[e]);
      if (st_out != nullptr) {
        st_out[0 * nBT + o + t] = Bc[e];
        st_out[1 * nBT + o + t] = Lc[e];
        st_out[2 * nBT + o + t] = Bd[e];
        st_out[3 * nBT + o + t] = Ld[e];
        if (t >= 1) {
          st_out[4 * nBT + o + t] = Bs[e];
          st_out[5 * nBT + o + t] = Ls[e];
        }
      }
    }
  }
}

// Plain generator prox: argmin c2 p^2 + c1 p + rho_hat/2 (p - X)^2 on [pmin, pmax].
template <typename R>
__device__ inline R gen_target(R X, R c1, R c2, R rho_hat) {
  return (rho_hat * X - c1) / (R(2) * c2 + rho_hat);
}


// Step 1 for one line and one 16-byte vector of contingencies (Section 4.2,
// DC line prox with the per-contingency susceptance and capacity of the N-1
// model), preceded by the deferred scaled-price update v += theta - thetabar
// of the previous iteration and the pending penalty rescale.  Both end
// nodes of a line call this with identical inputs.
template <typename R, int VEC>
struct LineOut {
  R p[VEC], tm[VEC], v1[VEC], v2[VEC], half[VEC];
  R u[VEC];  // unclipped flow target (0 for the outaged line)
};

template <typename R, typename VT, int VEC>
__device__ __forceinline__ void line_prox(const Vec<R, VEC>& P, const Vec<R, VEC>& Tm,
                                          const Vec<VT, VEC>& V1, const Vec<VT, VEC>& V2,
                                          const Vec<R, VEC>& Wf, const Vec<R, VEC>& Wh,
                                          const Vec<R, VEC>& Bf, const Vec<R, VEC>& Bh,
                                          const Vec<int32_t, VEC>& ok, int l, const R* td_old,
                                          int k0, int Kp, R inv2s, R cap, R rp, R rt, R sv,
                                          LineOut<R, VEC>& o) {
  // inv2s = 1 / (2 s), s the line's susceptance
  const R iden = R(1) / (R(2) * rp + R(2) * rt * inv2s * inv2s);  // 1 / (2 rho_p + rho_th / (2 s^2))
  const R ca = rp * iden;                                         // weight of z2 - z1
  const R cb = rt * inv2s * iden;                                 // weight of xi1 - xi2
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const bool outg = ok.x[e] == l;
    const R half = outg ? td_old[e] : P.x[e] * inv2s;
    const R th1 = Tm.x[e] + half, th2 = Tm.x[e] - half;
    R v1 = sv * (DIO<VT, R>::in(V1.x[e]) + th1 - Bf.x[e]);
    R v2 = sv * (DIO<VT, R>::in(V2.x[e]) + th2 - Bh.x[e]);
    const R z1 = -P.x[e] - Wf.x[e];  // ptilde - u at terminal 1 (p1 = -P)
    const R z2 = P.x[e] - Wh.x[e];   // ptilde - u at terminal 2
    const R xi1 = Bf.x[e] - v1, xi2 = Bh.x[e] - v2;
    R tm = R(0.5) * (xi1 + xi2);
    R pn, hn, u;
    if (outg) {
      u = pn = R(0);
      hn = R(0.5) * (xi1 - xi2);
    } else {
      u = ca * (z2 - z1) + cb * (xi1 - xi2);
      pn = clampv(u, -cap, cap);
      hn = pn * inv2s;
    }
    if (k0 + e >= Kp) pn = tm = v1 = v2 = hn = R(0);
    o.p[e] = pn;
    o.tm[e] = tm;
    o.v1[e] = v1;
    o.v2[e] = v2;
    o.half[e] = hn;
    o.u[e] = u;
  }
}

// General line model: the parameters of one line in each contingency of a
// 16-byte vector.  mode 0: AC line in service with susceptance s and
// capacity cap; 1: out of service (no power, both phases at their targets;
// the N-1 outage, or a change with zero susceptance); 2: HVDC link (Section
// 2.1: lossless transfer within cap, no phase relation).  hold: the stored
// half phase difference where it is not P/(2s) (modes 1 and 2); z: index of
// a change that takes the line out, whose half difference lives in Tz.
// line_prox with per-contingency parameters (the general line model).  The
// parameters of contingency k0+e are formed in the loop: the base values,
// the N-1 outage (ok), a DC link (dci >= 0; Hd: its stored half
// differences), then the line's changes (CSR entries ordered by
// contingency: a change sets a DC link's capacity, takes an AC line out
// (its stored half difference in tz_old[z]) or sets its susceptance and
// capacity).  td_old: the outaged lines' half differences for k0 ...
// k0+VEC-1.  With tz_new, the new half difference of a line a change takes
// out is stored at tz_new[z].
template <typename R, typename VT, int VEC>
__device__ __forceinline__ void line_prox_gen(const Topo& tp, int l, int k0,
                                              const Vec<int32_t, VEC>& ok, int dci,
                                              const Vec<R, VEC>& Hd, const R* td_old,
                                              const R* tz_old, R* tz_new, const Vec<R, VEC>& P,
                                              const Vec<R, VEC>& Tm, const Vec<VT, VEC>& V1,
                                              const Vec<VT, VEC>& V2, const Vec<R, VEC>& Wf,
                                              const Vec<R, VEC>& Wh, const Vec<R, VEC>& Bf,
                                              const Vec<R, VEC>& Bh, int Kp, R rp, R rt, R sv,
                                              LineOut<R, VEC>& o) {
  const R s0 = R(tp.sus[l]), cap0 = R(tp.cap[l]);
  const int c0 = tp.chg_ptr[l], c1 = tp.chg_ptr[l + 1];
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    const int k = k0 + e;
    const bool outg = ok.x[e] == l;
    R sus = s0, cap = cap0;
    int mode = outg ? 1 : (dci >= 0 ? 2 : 0), z = -1;
    R hold = dci >= 0 ? Hd.x[e] : (outg ? td_old[e] : R(0));
    for (int c = c0; c < c1; ++c) {
      const LineChg ch = tp.chg[c];
      if (ch.k > k) break;
      if (ch.k != k) continue;
      if (dci >= 0) {
        cap = R(ch.cap);
      } else if (ch.z >= 0) {
        mode = 1;
        z = ch.z;
        hold = tz_old[ch.z];
      } else {
        sus = R(ch.sus);
        cap = R(ch.cap);
      }
    }
    const R inv2s = R(0.5) / (mode == 0 ? sus : R(1));
    const R half = mode == 0 ? P.x[e] * inv2s : hold;
    const R th1 = Tm.x[e] + half, th2 = Tm.x[e] - half;
    R v1 = sv * (DIO<VT, R>::in(V1.x[e]) + th1 - Bf.x[e]);
    R v2 = sv * (DIO<VT, R>::in(V2.x[e]) + th2 - Bh.x[e]);
    const R z1 = -P.x[e] - Wf.x[e];
    const R z2 = P.x[e] - Wh.x[e];
    const R xi1 = Bf.x[e] - v1, xi2 = Bh.x[e] - v2;
    R tm = R(0.5) * (xi1 + xi2);
    R pn, hn, u;
    if (mode == 1) {
      u = pn = R(0);
      hn = R(0.5) * (xi1 - xi2);
    } else if (mode == 2) {  // HVDC link: flow at the clipped midpoint, phases at their targets
      u = R(0.5) * (z2 - z1);
      pn = clampv(u, -cap, cap);
      hn = R(0.5) * (xi1 - xi2);
    } else {
      const R iden = R(1) / (R(2) * rp + R(2) * rt * inv2s * inv2s);
      const R ca = rp * iden, cb = rt * inv2s * iden;
      u = ca * (z2 - z1) + cb * (xi1 - xi2);
      pn = clampv(u, -cap, cap);
      hn = pn * inv2s;
    }
    if (k >= Kp) pn = tm = v1 = v2 = hn = R(0);
    if (tz_new && z >= 0) tz_new[z] = hn;
    o.p[e] = pn;
    o.tm[e] = tm;
    o.v1[e] = v1;
    o.v2[e] = v2;
    o.half[e] = hn;
    o.u[e] = u;
  }
}

}  // namespace opf
