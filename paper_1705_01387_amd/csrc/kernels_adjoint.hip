// Reverse (adjoint) of the Chebyshev moment recurrence, for gradients of
// losses built on the moments of Section 3.3 with respect to the on-site
// energies and the hopping classes.
//
// Forward (Section 3.2): v_0 = phiR, v_1 = H~ v_0, v_n = 2 H~ v_{n-1} - v_{n-2},
// mu_n = <phiL|v_n>.  For L = sum_n w_n Re mu_n the adjoint vectors obey
//   lam_n = w_n phiL + 2 H~ lam_{n+1} - lam_{n+2},  lam_M = lam_{M+1} = 0,
// a Clenshaw-type recurrence run backwards, and
//   dL/dp = Re[ sum_{n>=2} 2 <lam_n| dH~/dp v_{n-1}> + <lam_1| dH~/dp v_0> ].
// With dH~/dU_i = e_i e_i^T / DeltaE and dH~/deps_c = H~_c (the class-c
// hoppings), one reverse step needs lam_{n+1} and v_{n-1} at the neighbours
// of each row: the kernel gathers both with the same neighbour indices, so a
// reverse step reads the matrix once.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace gpuqt {

using namespace dev;

namespace {

template <int B, int HOP, int K, int NC>
__global__ __launch_bounds__(kBlock) void k_adjoint_step(DevMat A, AdjIO io) {
  const int lb = logical_block(A.G);
  const BlkPlan P = A.plan[lb];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const double inv_dE = 1.0 / A.seg_dE[P.seg];
  const int b = threadIdx.x & (B - 1);
  // source coefficient of phiL: a real loss weight, or a complex series
  // coefficient J[seg][n] * src_phase (already conjugated by the caller)
  const double2 wn = io.Jtab ? cscale(io.Jtab[(int64_t)P.seg * io.ldJ + io.n], io.src_phase)
                             : make_double2(io.wts ? io.wts[((int64_t)P.seg * B + b) * io.M + io.n] : 0.0,
                                            0.0);
  const double2* __restrict__ x = io.x;
  const double2* __restrict__ v = io.v;
  const int S = 1 << A.S_log2;
  double gc[NC > 0 ? NC : 1];
#pragma unroll
  for (int c = 0; c < (NC > 0 ? NC : 1); ++c) gc[c] = 0.0;
  for_rows<B>(A, P, [&](int64_t r) {
    const int64_t idx = r * B + b;
    const int64_t sl = r >> A.S_log2;
    const int64_t p0 = A.slice_ptr[sl];
    const int64_t e0 = p0 + (r & (S - 1));
    const int w = K > 0 ? K : (int)((A.slice_ptr[sl + 1] - p0) >> A.S_log2);
    double2 h = make_double2(0.0, 0.0);
    double2 hv[NC > 0 ? NC : 1];
#pragma unroll
    for (int c = 0; c < (NC > 0 ? NC : 1); ++c) hv[c] = make_double2(0.0, 0.0);
    if (x) h = cscale(A.diag[r], x[idx]);
    for (int j = 0; j < w; ++j) {
      const int64_t e = e0 + (int64_t)j * S;
      int64_t cc;
      const bool ok = col_entry<HOP>(A, r, e, &cc);
      const double2 he = hop_entry<HOP>(A, e, ok, hu);
      if (x) {
        const double2 xv = x[cc * B + b];
        h = cadd(h, (HOP == HOP_COMPLEX || HOP == HOP_DICT) ? cmul(he, xv) : cscale(he.x, xv));
      }
      if (NC > 0 && v) {
        const double2 vv = v[cc * B + b];
        const double2 he0 = hop0_entry<HOP>(A, e, ok, P.seg);
        const double2 t = (HOP == HOP_COMPLEX || HOP == HOP_DICT) ? cmul(he0, vv) : cscale(he0.x, vv);
        const int cls = (NC > 1) ? (ok ? io.cls[HOP == HOP_DICT ? (int64_t)A.hidx[e] : e] : 0) : 0;
#pragma unroll
        for (int q = 0; q < (NC > 0 ? NC : 1); ++q)
          if (q == cls) hv[q] = cadd(hv[q], t);
      }
    }
    double2 lam = cmul(wn, io.phiL[idx]);
    lam = make_double2(fma(io.f_rec, h.x, lam.x), fma(io.f_rec, h.y, lam.y));
    if (io.w) {
      const double2 ww = io.w[idx];
      lam = make_double2(lam.x - ww.x, lam.y - ww.y);
    }
    io.out[idx] = io.accumulate ? cadd(io.out[idx], lam) : lam;
    if (v) {
      const double2 vr = v[idx];
      double gu = io.f * (lam.x * vr.x + lam.y * vr.y);     // f Re(conj(lam) v)
#pragma unroll
      for (int off = 1; off < B; off <<= 1) gu += __shfl_xor(gu, off);
      if (b == 0) io.gU[r] += gu * inv_dE;
#pragma unroll
      for (int q = 0; q < (NC > 0 ? NC : 1); ++q)
        if (NC > 0) gc[q] += io.f * (lam.x * hv[q].x + lam.y * hv[q].y);
      if (io.gH) row_entry_grads<B, HOP, K>(A, r, b, lam, v, io.f * inv_dE, io.gH, io.ldH);
    }
  });
  if (NC == 0 || !v) return;
  // class partials: workgroup sum in a fixed order, accumulated per workgroup
  __shared__ double sh[kBlock / 64][NC > 0 ? NC : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < (NC > 0 ? NC : 1); ++q) {
    double s = gc[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) sh[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < (NC > 0 ? NC : 1)) {
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < kBlock / 64; ++wv) s += sh[wv][threadIdx.x];
    io.gcp[(int64_t)lb * NC + threadIdx.x] += s;
  }
}

// Reverse step of the two-chain form (both adjoint chains in one launch, the
// matrix read once; abar_{k+1}, bbar_{k+1} and, for class gradients, a_{k-1},
// b_{k-1} gathered with the same indices).  Parameter terms, as for the
// single chain: dL/dp = Re sum_k f_k (<abar_k| dH~/dp a_{k-1}> + <bbar_k| dH~/dp b_{k-1}>).
template <int B, int HOP, int K, int NC>
__global__ __launch_bounds__(kBlock) void k_adjoint_pair_step(DevMat A, AdjPairIO io) {
  const int lb = logical_block(A.G);
  const BlkPlan P = A.plan[lb];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const double inv_dE = 1.0 / A.seg_dE[P.seg];
  const int b = threadIdx.x & (B - 1);
  const double* om = io.om + ((int64_t)P.seg * B + b) * io.R;
  const int k2 = 2 * io.k;
  const double w0 = om[k2];
  const double wm = io.k >= 1 ? om[k2 - 1] : 0.0;
  const double wp = (io.a_p1 && k2 + 1 < io.R) ? om[k2 + 1] : 0.0;
  const bool grad = io.gU != nullptr && io.k >= 1;
  const int S = 1 << A.S_log2;
  double gc[NC > 0 ? NC : 1];
#pragma unroll
  for (int c = 0; c < (NC > 0 ? NC : 1); ++c) gc[c] = 0.0;
  for_rows<B>(A, P, [&](int64_t r) {
    const int64_t idx = r * B + b;
    const int64_t sl = r >> A.S_log2;
    const int64_t p0 = A.slice_ptr[sl];
    const int64_t e0 = p0 + (r & (S - 1));
    const int w = K > 0 ? K : (int)((A.slice_ptr[sl + 1] - p0) >> A.S_log2);
    double2 ha = make_double2(0.0, 0.0), hb = make_double2(0.0, 0.0);
    double2 hva[NC > 0 ? NC : 1], hvb[NC > 0 ? NC : 1];
#pragma unroll
    for (int c = 0; c < (NC > 0 ? NC : 1); ++c) {
      hva[c] = make_double2(0.0, 0.0);
      hvb[c] = make_double2(0.0, 0.0);
    }
    if (io.xa) {
      const double d = A.diag[r];
      ha = cscale(d, io.xa[idx]);
      hb = cscale(d, io.xb[idx]);
    }
    for (int j = 0; j < w; ++j) {
      const int64_t e = e0 + (int64_t)j * S;
      int64_t cc;
      const bool ok = col_entry<HOP>(A, r, e, &cc);
      const double2 he = hop_entry<HOP>(A, e, ok, hu);
      if (io.xa) {
        const double2 xa = io.xa[cc * B + b], xb = io.xb[cc * B + b];
        ha = cadd(ha, (HOP == HOP_COMPLEX || HOP == HOP_DICT) ? cmul(he, xa) : cscale(he.x, xa));
        hb = cadd(hb, (HOP == HOP_COMPLEX || HOP == HOP_DICT) ? cmul(he, xb) : cscale(he.x, xb));
      }
      if (NC > 0 && grad) {
        const double2 va = io.a_m1[cc * B + b], vb = io.b_m1[cc * B + b];
        const double2 he0 = hop0_entry<HOP>(A, e, ok, P.seg);
        const double2 ta = (HOP == HOP_COMPLEX || HOP == HOP_DICT) ? cmul(he0, va) : cscale(he0.x, va);
        const double2 tb = (HOP == HOP_COMPLEX || HOP == HOP_DICT) ? cmul(he0, vb) : cscale(he0.x, vb);
        const int cls = (NC > 1) ? (ok ? io.cls[HOP == HOP_DICT ? (int64_t)A.hidx[e] : e] : 0) : 0;
#pragma unroll
        for (int q = 0; q < (NC > 0 ? NC : 1); ++q)
          if (q == cls) {
            hva[q] = cadd(hva[q], ta);
            hvb[q] = cadd(hvb[q], tb);
          }
      }
    }
    // direct sensitivities of the raw dots
    double2 ga = cscale(w0, io.b_k[idx]);
    if (io.k >= 1) ga = cadd(ga, cscale(wm, io.b_m1[idx]));
    double2 gb = cscale(w0, io.a_k[idx]);
    if (io.a_p1) gb = cadd(gb, cscale(wp, io.a_p1[idx]));
    double2 la = make_double2(fma(io.f_rec, ha.x, ga.x), fma(io.f_rec, ha.y, ga.y));
    double2 lbv = make_double2(fma(io.f_rec, hb.x, gb.x), fma(io.f_rec, hb.y, gb.y));
    if (io.wa) {
      const double2 u = io.wa[idx], v = io.wb[idx];
      la = make_double2(la.x - u.x, la.y - u.y);
      lbv = make_double2(lbv.x - v.x, lbv.y - v.y);
    }
    io.oa[idx] = io.acc_a ? cadd(io.oa[idx], la) : la;
    io.ob[idx] = io.acc_b ? cadd(io.ob[idx], lbv) : lbv;
    if (grad) {
      const double2 va = io.a_m1[idx], vb = io.b_m1[idx];
      double gu = io.f * (la.x * va.x + la.y * va.y + lbv.x * vb.x + lbv.y * vb.y);
#pragma unroll
      for (int off = 1; off < B; off <<= 1) gu += __shfl_xor(gu, off);
      if (b == 0) io.gU[r] += gu * inv_dE;
#pragma unroll
      for (int q = 0; q < (NC > 0 ? NC : 1); ++q)
        if (NC > 0)
          gc[q] += io.f * (la.x * hva[q].x + la.y * hva[q].y + lbv.x * hvb[q].x + lbv.y * hvb[q].y);
    }
  });
  if (NC == 0 || !grad) return;
  __shared__ double sh[kBlock / 64][NC > 0 ? NC : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < (NC > 0 ? NC : 1); ++q) {
    double s = gc[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) sh[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < (NC > 0 ? NC : 1)) {
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < kBlock / 64; ++wv) s += sh[wv][threadIdx.x];
    io.gcp[(int64_t)lb * NC + threadIdx.x] += s;
  }
}

// Reverse step of the Hermitian form (phiL = phiR, one chain a_k = T_k phi):
// with both chains equal the two adjoints only enter through their sum
// cbar_k = abar_k + bbar_k,
//   cbar_k = 2 om_2k a_k + om_2k-1 a_{k-1} + om_2k+1 a_{k+1} + f_rec H~ cbar_{k+1} - cbar_{k+2},
// and the parameter terms are Re sum_k f_k <cbar_k| dH~/dp a_{k-1}>: one chain
// gathered instead of two.  At k = 0 the output is cbar_0 / 2 = sum_n w_n T_n phi
// (abar_0 = bbar_0).  Fields of io: xa, wa, oa, acc_a, a_m1, a_k, a_p1 and the
// weights; the b fields are unused.
template <int B, int HOP, int K, int NC>
__global__ __launch_bounds__(kBlock) void k_adjoint_sym_step(DevMat A, AdjPairIO io) {
  const int lb = logical_block(A.G);
  const BlkPlan P = A.plan[lb];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const double inv_dE = 1.0 / A.seg_dE[P.seg];
  const int b = threadIdx.x & (B - 1);
  const double* om = io.om + ((int64_t)P.seg * B + b) * io.R;
  const int k2 = 2 * io.k;
  const double w0 = 2.0 * om[k2];
  const double wm = io.k >= 1 ? om[k2 - 1] : 0.0;
  const double wp = (io.a_p1 && k2 + 1 < io.R) ? om[k2 + 1] : 0.0;
  const double out_scale = io.k == 0 ? 0.5 : 1.0;
  const bool grad = io.gU != nullptr && io.k >= 1;
  const int S = 1 << A.S_log2;
  double gc[NC > 0 ? NC : 1];
#pragma unroll
  for (int c = 0; c < (NC > 0 ? NC : 1); ++c) gc[c] = 0.0;
  for_rows<B>(A, P, [&](int64_t r) {
    const int64_t idx = r * B + b;
    const int64_t sl = r >> A.S_log2;
    const int64_t p0 = A.slice_ptr[sl];
    const int64_t e0 = p0 + (r & (S - 1));
    const int w = K > 0 ? K : (int)((A.slice_ptr[sl + 1] - p0) >> A.S_log2);
    double2 h = make_double2(0.0, 0.0);
    double2 hv[NC > 0 ? NC : 1];
#pragma unroll
    for (int c = 0; c < (NC > 0 ? NC : 1); ++c) hv[c] = make_double2(0.0, 0.0);
    if (io.xa) h = cscale(A.diag[r], io.xa[idx]);
    for (int j = 0; j < w; ++j) {
      const int64_t e = e0 + (int64_t)j * S;
      int64_t cc;
      const bool ok = col_entry<HOP>(A, r, e, &cc);
      const double2 he = hop_entry<HOP>(A, e, ok, hu);
      if (io.xa) {
        const double2 x = io.xa[cc * B + b];
        h = cadd(h, (HOP == HOP_COMPLEX || HOP == HOP_DICT) ? cmul(he, x) : cscale(he.x, x));
      }
      if (NC > 0 && grad) {
        const double2 v = io.a_m1[cc * B + b];
        const double2 he0 = hop0_entry<HOP>(A, e, ok, P.seg);
        const double2 t = (HOP == HOP_COMPLEX || HOP == HOP_DICT) ? cmul(he0, v) : cscale(he0.x, v);
        const int cls = (NC > 1) ? (ok ? io.cls[HOP == HOP_DICT ? (int64_t)A.hidx[e] : e] : 0) : 0;
#pragma unroll
        for (int q = 0; q < (NC > 0 ? NC : 1); ++q)
          if (q == cls) hv[q] = cadd(hv[q], t);
      }
    }
    // direct sensitivities of the raw dots
    double2 g = cscale(w0, io.a_k[idx]);
    if (io.k >= 1) g = cadd(g, cscale(wm, io.a_m1[idx]));
    if (io.a_p1) g = cadd(g, cscale(wp, io.a_p1[idx]));
    double2 c = make_double2(fma(io.f_rec, h.x, g.x), fma(io.f_rec, h.y, g.y));
    if (io.wa) {
      const double2 u = io.wa[idx];
      c = make_double2(c.x - u.x, c.y - u.y);
    }
    const double2 o = cscale(out_scale, c);
    io.oa[idx] = io.acc_a ? cadd(io.oa[idx], o) : o;
    if (grad) {
      const double2 v = io.a_m1[idx];
      double gu = io.f * (c.x * v.x + c.y * v.y);
#pragma unroll
      for (int off = 1; off < B; off <<= 1) gu += __shfl_xor(gu, off);
      if (b == 0) io.gU[r] += gu * inv_dE;
#pragma unroll
      for (int q = 0; q < (NC > 0 ? NC : 1); ++q)
        if (NC > 0) gc[q] += io.f * (c.x * hv[q].x + c.y * hv[q].y);
    }
  });
  if (NC == 0 || !grad) return;
  __shared__ double sh[kBlock / 64][NC > 0 ? NC : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < (NC > 0 ? NC : 1); ++q) {
    double s = gc[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) sh[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < (NC > 0 ? NC : 1)) {
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < kBlock / 64; ++wv) s += sh[wv][threadIdx.x];
    io.gcp[(int64_t)lb * NC + threadIdx.x] += s;
  }
}

// Raw-dot weights of the product identities, one wavefront per (segment,
// column) row: lane l sums w_n for n = 2 + l + 64 j (all of one parity, the
// parity of l), a butterfly over lanes of equal parity gives the even and odd
// tails in a fixed order, and the lanes write om[n] for n = l, l + 64, ...
__global__ __launch_bounds__(64) void k_raw_weights(const double* __restrict__ w, int M, int R,
                                                    double* __restrict__ om) {
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  const double* wi = w + i * M;
  double* oi = om + i * R;
  double t = 0.0;
  for (int n = 2 + lane; n < M; n += 64) t += wi[n];
#pragma unroll
  for (int off = 2; off < 64; off <<= 1) t += __shfl_xor(t, off);
  const double even = __shfl(t, 0), odd = __shfl(t, 1);
  for (int n = lane; n < R; n += 64) {
    double v = 0.0;
    if (n == 0) v = (M > 0 ? wi[0] : 0.0) - even;
    else if (n == 1) v = (M > 1 ? wi[1] : 0.0) - odd;
    else if (n < M) v = 2.0 * wi[n];
    oi[n] = v;
  }
}

// gcp[lb][c] += Re sum_i conj(a_i) (V_c x)_i over the workgroup's rows, with
// V_c = i dx H_c the velocity restricted to the class-c hoppings (unscaled:
// the stored H~ is multiplied back by DeltaE).
template <int B, int HOP, int NC>
__global__ __launch_bounds__(kBlock) void k_velocity_class_grad(DevMat A, const double2* __restrict__ a,
                                                                const double2* __restrict__ x,
                                                                const int32_t* __restrict__ cls,
                                                                double* __restrict__ gcp) {
  const int lb = logical_block(A.G);
  const BlkPlan P = A.plan[lb];
  const double e = A.seg_dE[P.seg];
  const int b = threadIdx.x & (B - 1);
  const int S = 1 << A.S_log2;
  double gc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) gc[q] = 0.0;
  for_rows<B>(A, P, [&](int64_t r) {
    const int64_t idx = r * B + b;
    const int64_t sl = r >> A.S_log2;
    const int64_t p0 = A.slice_ptr[sl];
    const int64_t e0 = p0 + (r & (S - 1));
    const int w = (int)((A.slice_ptr[sl + 1] - p0) >> A.S_log2);
    const double2 ar = a[idx];
    for (int j = 0; j < w; ++j) {
      const int64_t en = e0 + (int64_t)j * S;
      int64_t c;
      if (!col_entry<HOP>(A, r, en, &c)) continue;
      const double2 he = hop0_entry<HOP>(A, en, true, P.seg);
      const double2 t = cmul(he, x[c * B + b]);
      const double s = e * dx_entry<HOP>(A, en);
      const double2 vt = make_double2(-s * t.y, s * t.x);      // i e dx H~ x
      const double contrib = ar.x * vt.x + ar.y * vt.y;        // Re conj(a) vt
      const int q0 = (NC > 1) ? cls[HOP == HOP_DICT ? (int64_t)A.hidx[en] : en] : 0;
#pragma unroll
      for (int q = 0; q < NC; ++q)
        if (q == q0) gc[q] += contrib;
    }
  });
  __shared__ double sh[kBlock / 64][NC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    double s = gc[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) sh[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < NC) {
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < kBlock / 64; ++wv) s += sh[wv][threadIdx.x];
    gcp[(int64_t)lb * NC + threadIdx.x] += s;
  }
}

// Per-entry share of a^+ V x, V_ij = i dx_ij H_ij (unscaled):
// g_ij = i dx_ij sum_b conj(a_ib) x_jb, gH[i*ldH + slot] += (Re g, -Im g).
template <int B, int HOP>
__global__ __launch_bounds__(kBlock) void k_velocity_entry_grad(DevMat A, const double2* __restrict__ a,
                                                                const double2* __restrict__ x,
                                                                double* __restrict__ gH, int ldH) {
  const BlkPlan P = A.plan[logical_block(A.G)];
  const int b = threadIdx.x & (B - 1);
  const int S = 1 << A.S_log2;
  for_rows<B>(A, P, [&](int64_t r) {
    const double2 ar = a[r * B + b];
    const int64_t sl = r >> A.S_log2;
    const int64_t p0 = A.slice_ptr[sl];
    const int64_t e0 = p0 + (r & (S - 1));
    const int w = (int)((A.slice_ptr[sl + 1] - p0) >> A.S_log2);
    for (int j = 0; j < w; ++j) {
      const int64_t en = e0 + (int64_t)j * S;
      int64_t c;
      const bool ok = col_entry<HOP>(A, r, en, &c);
      const double2 xv = x[c * B + b];
      double zr = ar.x * xv.x + ar.y * xv.y;   // z = conj(a) x
      double zi = ar.x * xv.y - ar.y * xv.x;
      zr = row_lanes_sum<B>(zr);
      zi = row_lanes_sum<B>(zi);
      if (ok && b == 0) {
        const double d = dx_entry<HOP>(A, en);   // g = i d z: (Re g, -Im g) = (-d Im z, -d Re z)
        double* p = gH + 2 * (r * (int64_t)ldH + j);
        p[0] -= d * zi;
        p[1] -= d * zr;
      }
    }
  });
}

// Hermitian tie of per-entry gradients, one thread per (row i, slot s): entry
// (i, s) -> j is the q-th of row i's entries pointing to j; its partner is the
// q-th entry of row j pointing to i.  out = (re_is + re_jp, im_is - im_jp), or
// the entry's own value without a partner (and for padding slots).
template <int HOP>
__global__ __launch_bounds__(256) void k_tie_entries(DevMat A, int64_t n, int ldH, const double* __restrict__ in,
                                                     double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ldH) return;
  const int64_t i = t / ldH;
  const int s = (int)(t - i * ldH);
  const int S = 1 << A.S_log2;
  auto width = [&](int64_t r) { const int64_t sl = r >> A.S_log2; return (int)((A.slice_ptr[sl + 1] - A.slice_ptr[sl]) >> A.S_log2); };
  auto entry = [&](int64_t r, int j) { return A.slice_ptr[r >> A.S_log2] + (int64_t)j * S + (r & (S - 1)); };
  double re = in[2 * t], im = in[2 * t + 1];
  int64_t j = -1;
  if (s < width(i)) {
    int64_t c;
    if (col_entry<HOP>(A, i, entry(i, s), &c)) j = c;
  }
  if (j >= 0) {
    int q = 0;
    for (int u = 0; u < s; ++u) {
      int64_t c;
      if (col_entry<HOP>(A, i, entry(i, u), &c) && c == j) ++q;
    }
    const int wj = width(j);
    for (int u = 0; u < wj && u < ldH; ++u) {
      int64_t c;
      if (col_entry<HOP>(A, j, entry(j, u), &c) && c == i) {
        if (q == 0) {
          re += in[2 * (j * ldH + u)];
          im -= in[2 * (j * ldH + u) + 1];
          break;
        }
        --q;
      }
    }
  }
  out[2 * t] = re;
  out[2 * t + 1] = im;
}

// diag[r] = onsite[r] / DeltaE_seg (new on-site energies)
__global__ __launch_bounds__(kBlock) void k_set_onsite(DevMat A, const double* __restrict__ onsite,
                                                       double* __restrict__ diag) {
  const BlkPlan P = A.plan[logical_block(A.G)];
  const double inv = 1.0 / A.seg_dE[P.seg];
  for_rows<1>(A, P, [&](int64_t r) { diag[r] = onsite[r] * inv; });
}

// hop[e] = hop0[e] * scale[class of e]  (real: one double per entry, complex: two)
__global__ __launch_bounds__(256) void k_scale_hops(int64_t entries, int cplx, const double* __restrict__ hop0,
                                                    double* __restrict__ hop, const int32_t* __restrict__ cls,
                                                    ClassScale sc) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < entries;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = cls ? cls[e] : 0;
    const double f = c >= 0 ? sc.s[c] : 0.0;
    if (cplx) {
      hop[2 * e] = hop0[2 * e] * f;
      hop[2 * e + 1] = hop0[2 * e + 1] * f;
    } else {
      hop[e] = hop0[e] * f;
    }
  }
}

// bound[lb] = max over the workgroup's rows of |U~_r| + sum_j |H~_rj| (the
// Gershgorin bound of H / DeltaE, which must stay <= 1)
template <int HOP>
__global__ __launch_bounds__(kBlock) void k_row_bound(DevMat A, double* __restrict__ bound) {
  const int lb = logical_block(A.G);
  const BlkPlan P = A.plan[lb];
  const double hu = (HOP == HOP_UNIFORM) ? fabs(A.seg_hop[P.seg]) : 0.0;
  const int S = 1 << A.S_log2;
  double mx = 0.0;
  for_rows<1>(A, P, [&](int64_t r) {
    const int64_t sl = r >> A.S_log2;
    const int64_t p0 = A.slice_ptr[sl];
    const int64_t e0 = p0 + (r & (S - 1));
    const int w = (int)((A.slice_ptr[sl + 1] - p0) >> A.S_log2);
    double s = fabs(A.diag[r]);
    for (int j = 0; j < w; ++j) {
      const int64_t e = e0 + (int64_t)j * S;
      int64_t c;
      if (!col_entry<HOP>(A, r, e, &c)) continue;
      const double2 he = hop_entry<HOP>(A, e, true, hu);
      s += HOP == HOP_UNIFORM ? hu : (HOP == HOP_REAL ? fabs(he.x) : hypot(he.x, he.y));
    }
    mx = fmax(mx, s);
  });
  __shared__ double sh[kBlock / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) m = fmax(m, sh[q]);
    bound[lb] = m;
  }
}

__global__ __launch_bounds__(256) void k_zero(double* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// grad_class[c] += sum over workgroups of gcp[g][c], in a fixed order.
__global__ __launch_bounds__(64) void k_reduce_classes(const double* __restrict__ gcp, int G, int NC,
                                                       double* __restrict__ out) {
  const int c = blockIdx.x;
  double s = 0.0;
  for (int g = threadIdx.x; g < G; g += 64) s += gcp[(int64_t)g * NC + c];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (threadIdx.x == 0) out[c] += s;
}

}  // namespace

hipError_t launch_adjoint_step(const DevMat& A, int hop_mode, int B, int nc, const AdjIO& io,
                               hipStream_t s) {
  return dispatch_bh(B, hop_mode, [&](auto Bc, auto Hc) {
    constexpr int Bv = decltype(Bc)::value, Hv = decltype(Hc)::value;
    auto go = [&](auto Kc) {
      constexpr int Kv = decltype(Kc)::value;
      switch (nc) {
        case 0: k_adjoint_step<Bv, Hv, Kv, 0><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
        case 1: k_adjoint_step<Bv, Hv, Kv, 1><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
        case 2: k_adjoint_step<Bv, Hv, Kv, 2><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
        default: k_adjoint_step<Bv, Hv, Kv, 4><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
      }
    };
    switch (A.K) {
      case 3: go(IC<3>{}); break;
      case 4: go(IC<4>{}); break;
      case 6: go(IC<6>{}); break;
      case 8: go(IC<8>{}); break;
      default: go(IC<0>{}); break;
    }
  });
}

hipError_t launch_adjoint_pair_step(const DevMat& A, int hop_mode, int B, int nc, const AdjPairIO& io,
                                    hipStream_t s) {
  return dispatch_bh(B, hop_mode, [&](auto Bc, auto Hc) {
    constexpr int Bv = decltype(Bc)::value, Hv = decltype(Hc)::value;
    auto go = [&](auto Kc) {
      constexpr int Kv = decltype(Kc)::value;
      switch (nc) {
        case 0: k_adjoint_pair_step<Bv, Hv, Kv, 0><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
        case 1: k_adjoint_pair_step<Bv, Hv, Kv, 1><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
        case 2: k_adjoint_pair_step<Bv, Hv, Kv, 2><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
        default: k_adjoint_pair_step<Bv, Hv, Kv, 4><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
      }
    };
    switch (A.K) {
      case 3: go(IC<3>{}); break;
      case 4: go(IC<4>{}); break;
      case 6: go(IC<6>{}); break;
      case 8: go(IC<8>{}); break;
      default: go(IC<0>{}); break;
    }
  });
}

hipError_t launch_adjoint_sym_step(const DevMat& A, int hop_mode, int B, int nc, const AdjPairIO& io,
                                   hipStream_t s) {
  return dispatch_bh(B, hop_mode, [&](auto Bc, auto Hc) {
    constexpr int Bv = decltype(Bc)::value, Hv = decltype(Hc)::value;
    auto go = [&](auto Kc) {
      constexpr int Kv = decltype(Kc)::value;
      switch (nc) {
        case 0: k_adjoint_sym_step<Bv, Hv, Kv, 0><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
        case 1: k_adjoint_sym_step<Bv, Hv, Kv, 1><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
        case 2: k_adjoint_sym_step<Bv, Hv, Kv, 2><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
        default: k_adjoint_sym_step<Bv, Hv, Kv, 4><<<dim3(A.G), kBlock, 0, s>>>(A, io); break;
      }
    };
    switch (A.K) {
      case 3: go(IC<3>{}); break;
      case 4: go(IC<4>{}); break;
      case 6: go(IC<6>{}); break;
      case 8: go(IC<8>{}); break;
      default: go(IC<0>{}); break;
    }
  });
}

hipError_t launch_raw_weights(const double* w, int rows, int M, int R, double* om, hipStream_t s) {
  if (rows <= 0 || R <= 0) return hipSuccess;
  k_raw_weights<<<dim3(rows), 64, 0, s>>>(w, M, R, om);
  return hipGetLastError();
}

hipError_t launch_velocity_class_grad(const DevMat& A, int hop_mode, int B, int nc, const double2* a,
                                      const double2* x, const int32_t* cls, double* gcp, hipStream_t s) {
  return dispatch_bh(B, hop_mode, [&](auto Bc, auto Hc) {
    constexpr int Bv = decltype(Bc)::value, Hv = decltype(Hc)::value;
    switch (nc) {
      case 1: k_velocity_class_grad<Bv, Hv, 1><<<dim3(A.G), kBlock, 0, s>>>(A, a, x, cls, gcp); break;
      case 2: k_velocity_class_grad<Bv, Hv, 2><<<dim3(A.G), kBlock, 0, s>>>(A, a, x, cls, gcp); break;
      default: k_velocity_class_grad<Bv, Hv, 4><<<dim3(A.G), kBlock, 0, s>>>(A, a, x, cls, gcp); break;
    }
  });
}

hipError_t launch_velocity_entry_grad(const DevMat& A, int hop_mode, int B, const double2* a, const double2* x,
                                      double* gH, int ldH, hipStream_t s) {
  return dispatch_bh(B, hop_mode, [&](auto Bc, auto Hc) {
    k_velocity_entry_grad<decltype(Bc)::value, decltype(Hc)::value><<<dim3(A.G), kBlock, 0, s>>>(A, a, x, gH,
                                                                                                  ldH);
  });
}

hipError_t launch_tie_entries(const DevMat& A, int hop_mode, int64_t n, int ldH, const double* in, double* out,
                              hipStream_t s) {
  const int64_t total = n * (int64_t)ldH;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks);
  if (hop_mode == HOP_UNIFORM) k_tie_entries<HOP_UNIFORM><<<g, 256, 0, s>>>(A, n, ldH, in, out);
  else if (hop_mode == HOP_REAL) k_tie_entries<HOP_REAL><<<g, 256, 0, s>>>(A, n, ldH, in, out);
  else if (hop_mode == HOP_COMPLEX) k_tie_entries<HOP_COMPLEX><<<g, 256, 0, s>>>(A, n, ldH, in, out);
  else k_tie_entries<HOP_DICT><<<g, 256, 0, s>>>(A, n, ldH, in, out);
  return hipGetLastError();
}

hipError_t launch_set_onsite(const DevMat& A, const double* onsite, double* diag, hipStream_t s) {
  k_set_onsite<<<dim3(A.G), kBlock, 0, s>>>(A, onsite, diag);
  return hipGetLastError();
}

hipError_t launch_scale_hops(int64_t entries, int cplx, const double* hop0, double* hop,
                             const int32_t* cls, const ClassScale& sc, hipStream_t s) {
  if (entries <= 0) return hipSuccess;
  int64_t blocks = (entries + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_scale_hops<<<dim3((unsigned)blocks), 256, 0, s>>>(entries, cplx, hop0, hop, cls, sc);
  return hipGetLastError();
}

hipError_t launch_row_bound(const DevMat& A, int hop_mode, double* bound, hipStream_t s) {
  if (hop_mode == HOP_UNIFORM) k_row_bound<HOP_UNIFORM><<<dim3(A.G), kBlock, 0, s>>>(A, bound);
  else if (hop_mode == HOP_REAL) k_row_bound<HOP_REAL><<<dim3(A.G), kBlock, 0, s>>>(A, bound);
  else if (hop_mode == HOP_COMPLEX) k_row_bound<HOP_COMPLEX><<<dim3(A.G), kBlock, 0, s>>>(A, bound);
  else k_row_bound<HOP_DICT><<<dim3(A.G), kBlock, 0, s>>>(A, bound);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_zero<<<dim3((unsigned)blocks), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_reduce_classes(const double* gcp, int G, int nc, int n_out, double* out, hipStream_t s) {
  if (nc <= 0 || n_out <= 0) return hipSuccess;
  k_reduce_classes<<<dim3(n_out), 64, 0, s>>>(gcp, G, nc, out);
  return hipGetLastError();
}

}  // namespace gpuqt
