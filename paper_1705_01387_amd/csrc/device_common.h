// Device helpers shared by the sparse kernels (kernels.hip, kernels_adjoint.hip):
// complex FP64 arithmetic, the row product over the sliced-ELL layout, the
// XCD-aware row schedule, the deterministic workgroup reduction and the
// compile-time dispatch over (B, hopping mode, row width, load variant).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace gpuqt {
namespace dev {

template <int V>
using IC = std::integral_constant<int, V>;

typedef double d2v __attribute__((ext_vector_type(2)));

template <bool NT, typename T>
__device__ __forceinline__ T ldg(const T* p) {
  if constexpr (NT) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}

template <bool NT>
__device__ __forceinline__ double2 ld2(const double2* p) {
  if constexpr (NT) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
    return make_double2(v.x, v.y);
  } else {
    return *p;
  }
}

__device__ __forceinline__ int logical_block(int G) {
  const int p = blockIdx.x;
  if ((G & 7) == 0) {
    const int per = G >> 3;
    return (p & 7) * per + (p >> 3);
  }
  return p;
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// a * b (complex)
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// 2 a - w
__device__ __forceinline__ double2 twice_minus(double2 a, double2 w) {
  return make_double2(fma(2.0, a.x, -w.x), fma(2.0, a.y, -w.y));
}
// acc += conj(a) * b
__device__ __forceinline__ void cdot_acc(double& re, double& im, double2 a, double2 b) {
  re = fma(a.x, b.x, fma(a.y, b.y, re));
  im = fma(a.x, b.y, fma(-a.y, b.x, im));
}

// Hopping H~ of entry e (ok: not padding) and its position difference, for
// every storage mode.
template <int HOP, bool NT = false>
__device__ __forceinline__ double2 hop_entry(const DevMat& A, int64_t e, bool ok, double hu) {
  if constexpr (HOP == HOP_UNIFORM) {
    return make_double2(ok ? hu : 0.0, 0.0);
  } else if constexpr (HOP == HOP_REAL) {
    return make_double2(ldg<NT>(A.hop + e), 0.0);
  } else if constexpr (HOP == HOP_COMPLEX) {
    return ld2<NT>(reinterpret_cast<const double2*>(A.hop) + e);
  } else {
    return A.htab[ldg<NT>(A.hidx + e)];
  }
}
// The build-time hopping of entry e (before class scales): class gradients are
// derivatives with respect to the scale s_c of H_c = s_c x (build-time H_c).
template <int HOP>
__device__ __forceinline__ double2 hop0_entry(const DevMat& A, int64_t e, bool ok, int seg) {
  if constexpr (HOP == HOP_UNIFORM) {
    return make_double2(ok ? A.seg_hop0[seg] : 0.0, 0.0);
  } else if constexpr (HOP == HOP_REAL) {
    return make_double2(A.hop0[e], 0.0);
  } else if constexpr (HOP == HOP_COMPLEX) {
    return reinterpret_cast<const double2*>(A.hop0)[e];
  } else {
    return A.htab0[A.hidx[e]];
  }
}
template <int HOP, bool NT = false>
__device__ __forceinline__ double dx_entry(const DevMat& A, int64_t e) {
  if constexpr (HOP == HOP_DICT) {
    return A.dxtab[ldg<NT>(A.hidx + e)];
  } else {
    return ldg<NT>(A.dx + e);
  }
}
// Column of entry e of row r: false for padding (then *cc = r, the hopping is 0).
template <int HOP>
__device__ __forceinline__ bool col_entry(const DevMat& A, int64_t r, int64_t e, int64_t* cc) {
  if constexpr (HOP == HOP_DICT) {
    const uint32_t id = A.hidx[e];
    *cc = r + A.offtab[id];
    return id != 0;
  } else {
    const int32_t c = A.col[e];
    *cc = c >= 0 ? (int64_t)c : r;
    return c >= 0;
  }
}

// Products of one row with the gathered vector(s):
//   ha = sum_j H~_rj xa_j (+ H~_rr xa_r),  hb likewise for xb (TWO),
//   da = sum_j dx_rj H~_rj xa_j (DX; the diagonal has dx = 0).
// xra / xrb are the row's own elements xa_r / xb_r, loaded by the caller
// together with its other per-row operands, so that every load that does not
// depend on a column index is in flight before the index loads return.
// K > 0: every slice has exactly K entries per row, so the row's first entry
// follows from r alone (no slice-offset load) and the loop is fully unrolled
// with all index loads issued before the gathers.  K == 0: runtime slice width.
// pk (K > 0 only): the row's keys, already loaded by for_rows_pf one tile
// ahead (NULL: load them here).
template <int B, int HOP, int K, bool NT, bool TWO, bool DX, bool DIAG>
__device__ __forceinline__ void row_apply(const DevMat& A, int64_t r, int b, double hu,
                                          const double2* __restrict__ xa,
                                          const double2* __restrict__ xb, double2 xra, double2 xrb,
                                          double2& ha, double2& hb, double2& da,
                                          const int32_t* pk = nullptr) {
  const int S = 1 << A.S_log2;
  const int64_t sl = r >> A.S_log2;
  const int64_t e0 = (K > 0 ? sl * ((int64_t)K << A.S_log2) : A.slice_ptr[sl]) + (r & (S - 1));
  ha = make_double2(0.0, 0.0);
  hb = make_double2(0.0, 0.0);
  da = make_double2(0.0, 0.0);
  if (DIAG) {
    const double d = ldg<NT>(A.diag + r);
    ha = cscale(d, xra);
    if (TWO) hb = cscale(d, xrb);
  }
  // key of an entry: its column (-1: padding), or (HOP_DICT) its table index,
  // whose entry holds the column offset, the hopping and dx (index 0: padding)
  auto key_at = [&](int64_t e) -> int32_t {
    if constexpr (HOP == HOP_DICT) {
      return (int32_t)ldg<NT>(A.hidx + e);
    } else {
      return ldg<NT>(A.col + e);
    }
  };
  auto body = [&](int32_t key, int64_t e) {
    constexpr bool CPLX = HOP == HOP_COMPLEX || HOP == HOP_DICT;
    double2 h;
    double dxv = 0.0;
    int64_t cc;
    if constexpr (HOP == HOP_DICT) {
      cc = r + A.offtab[key];
      h = A.htab[key];
      if (DX) dxv = A.dxtab[key];
    } else {
      const bool ok = key >= 0;
      cc = ok ? (int64_t)key : r;
      h = hop_entry<HOP, NT>(A, e, ok, hu);
      if (DX) dxv = ldg<NT>(A.dx + e);
    }
    const double2 v = xa[cc * B + b];
    const double2 hv = CPLX ? cmul(h, v) : cscale(h.x, v);
    ha = cadd(ha, hv);
    if (TWO) {
      const double2 u = xb[cc * B + b];
      hb = cadd(hb, CPLX ? cmul(h, u) : cscale(h.x, u));
    }
    if (DX) da = make_double2(fma(dxv, hv.x, da.x), fma(dxv, hv.y, da.y));
  };
  if constexpr (K > 0) {
    int32_t c[K];
#pragma unroll
    for (int j = 0; j < K; ++j) c[j] = pk ? pk[j] : key_at(e0 + (int64_t)j * S);
#pragma unroll
    for (int j = 0; j < K; ++j) body(c[j], e0 + (int64_t)j * S);
  } else {
    const int w = (int)((A.slice_ptr[sl + 1] - A.slice_ptr[sl]) >> A.S_log2);
    int j = 0;
    for (; j + 4 <= w; j += 4) {
      int32_t c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) c[q] = key_at(e0 + (int64_t)(j + q) * S);
#pragma unroll
      for (int q = 0; q < 4; ++q) body(c[q], e0 + (int64_t)(j + q) * S);
    }
    for (; j < w; ++j) body(key_at(e0 + (int64_t)j * S), e0 + (int64_t)j * S);
  }
}

// Visit the rows of this workgroup in tiles of RPI = 256/B rows: tiles j,
// j + g, j + 2g, ... of its group's row sequence (the contiguous range
// [r0, r1), or the units u0 .. u0 + nu of the banded or pencil order when the
// view has one).  f(r) for each row r of the thread; all threads of the
// workgroup iterate the same number of times.
template <int B, typename F>
__device__ __forceinline__ void for_rows(const DevMat& A, const BlkPlan& P, F&& f) {
  constexpr int RPI = kBlock / B;
  const int64_t step = (int64_t)P.g * RPI;
  if (A.pencil) {   // the same rule as row_at_pencil, per tile t
    constexpr int RPW = 64 / B;
    const int64_t total = pencil_seq_len(P);
    const int32_t* __restrict__ units = A.units + P.u0;
    const int w = threadIdx.x >> 6, l = (threadIdx.x & 63) / B;
    for (int64_t t = P.j; t * RPI < total; t += P.g) {
      const int64_t u = (t / B) * kPencil + w;
      if (u < P.nu) {
        const int64_t a = units[u];
        const int64_t r = a + (t % B) * RPW + l;
        if (r < (((a >> kUnitLog2) + 1) << kUnitLog2) && r < P.se) f(r);
      }
    }
    return;
  }
  if (A.units == nullptr) {   // linear: the same rule as row_at, without the call
    for (int64_t base = P.r0 + (int64_t)P.j * RPI; base < P.r1; base += step) {
      const int64_t r = base + threadIdx.x / B;
      if (r < P.r1) f(r);
    }
    return;
  }
  // banded: the same rule as row_at, with the unit start of the next tile
  // loaded one iteration ahead so that the lookup is off the row's load chain
  const int64_t total = row_seq_len(P, A.units);
  const int32_t* __restrict__ units = A.units + P.u0;
  int64_t pos = (int64_t)P.j * RPI + threadIdx.x / B;
  int32_t a_next = pos < total ? units[pos >> kUnitLog2] : 0;
  for (int64_t pos0 = (int64_t)P.j * RPI; pos0 < total; pos0 += step, pos += step) {
    const int64_t a = a_next;
    if (pos + step < total) a_next = units[(pos + step) >> kUnitLog2];
    if (pos < total) {
      const int64_t r = a + (pos & ((int64_t(1) << kUnitLog2) - 1));
      if (r < (((a >> kUnitLog2) + 1) << kUnitLog2) && r < P.se) f(r);
    }
  }
}

// Keys of the K entries of row r (fixed slice width K): column indices, or
// (HOP_DICT) table indices.
template <int HOP, int K, bool NT>
__device__ __forceinline__ void load_keys(const DevMat& A, int64_t r, int32_t* k) {
  const int S = 1 << A.S_log2;
  const int64_t e0 = (r >> A.S_log2) * ((int64_t)K << A.S_log2) + (r & (S - 1));
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if constexpr (HOP == HOP_DICT) {
      k[j] = (int32_t)ldg<NT>(A.hidx + e0 + (int64_t)j * S);
    } else {
      k[j] = ldg<NT>(A.col + e0 + (int64_t)j * S);
    }
  }
}

// The keys of row r split over the row's B lanes: lane b loads keys b, b + B,
// b + 2B, ... (k[i] = key b + i B, 0 past K), so a row's keys cost ceil(K / B)
// load instructions per wavefront instead of K; expand_keys gathers them back.
template <int HOP, int K, int B, bool NT>
__device__ __forceinline__ void load_keys_split(const DevMat& A, int64_t r, int32_t* k) {
  if constexpr (B == 1) {
    load_keys<HOP, K, NT>(A, r, k);
  } else {
    const int b = threadIdx.x & (B - 1);
    const int S = 1 << A.S_log2;
    const int64_t e0 = (r >> A.S_log2) * ((int64_t)K << A.S_log2) + (r & (S - 1));
#pragma unroll
    for (int i = 0; i < (K + B - 1) / B; ++i) {
      const int j = b + i * B;
      k[i] = 0;
      if (j < K) {
        if constexpr (HOP == HOP_DICT) {
          k[i] = (int32_t)ldg<NT>(A.hidx + e0 + (int64_t)j * S);
        } else {
          k[i] = ldg<NT>(A.col + e0 + (int64_t)j * S);
        }
      }
    }
  }
}
// All K keys of the row from the split of load_keys_split: key j sits in lane
// j mod B of the row's lanes, in its register j / B.  Every lane of the row must
// take part (cross-lane reads).
template <int K, int B>
__device__ __forceinline__ void expand_keys(const int32_t* kl, int32_t* keys) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if constexpr (B == 1) {
      keys[j] = kl[j];
    } else {
      keys[j] = __shfl(kl[j / B], j % B, B);
    }
  }
}

// The rows of for_rows, with the keys of each thread's next row loaded while
// the current row is processed: f(r, keys) gets keys already in registers, so
// a row waits for one memory trip (its gathers, issued together with its own
// per-row loads) instead of two (keys, then gathers).  Lanes past the end
// prefetch the keys of a valid row (the last row of the range, or the start
// of the unit) and discard them.  K == 0 (runtime slice widths): for_rows with
// keys = NULL.
template <int B, int HOP, int K, bool NT, typename F>
__device__ __forceinline__ void for_rows_pf(const DevMat& A, const BlkPlan& P, F&& f) {
  if constexpr (K == 0) {
    for_rows<B>(A, P, [&](int64_t r) { f(r, (const int32_t*)nullptr); });
  } else {
    constexpr int RPI = kBlock / B;
    constexpr int KL = (K + B - 1) / B;   // keys each lane loads
    const int64_t step = (int64_t)P.g * RPI;
    int32_t kc[KL], kn[KL];
    auto ldk = [&](int64_t r, int32_t* k) { load_keys_split<HOP, K, B, NT>(A, r, k); };
    // expand the row's keys (every lane of the workgroup takes part), then f for a valid row
    auto run = [&](int64_t r, bool ok) {
      int32_t keys[K];
      expand_keys<K, B>(kc, keys);
      if (ok) f(r, (const int32_t*)keys);
    };
    if (A.units == nullptr) {
      if (P.r1 <= P.r0) return;
      const int64_t last = P.r1 - 1;
      int64_t r = P.r0 + (int64_t)P.j * RPI + threadIdx.x / B;
      ldk(r < last ? r : last, kc);
      for (int64_t base = P.r0 + (int64_t)P.j * RPI; base < P.r1; base += step, r += step) {
        const int64_t rn = r + step;
        ldk(rn < last ? rn : last, kn);
        run(r, r < P.r1);
#pragma unroll
        for (int j = 0; j < KL; ++j) kc[j] = kn[j];
      }
      return;
    }
    if (A.pencil) {
      // pencil: per tile t the unit of this wavefront (row_at_pencil); unit
      // starts two tiles ahead, keys one tile ahead
      constexpr int RPW = 64 / B;
      const int64_t total = pencil_seq_len(P);
      if (total <= 0) return;
      const int32_t* __restrict__ units = A.units + P.u0;
      const int w = threadIdx.x >> 6, l = (threadIdx.x & 63) / B;
      const int64_t g = P.g, nu = P.nu;
      auto unit_of = [&](int64_t t) -> int64_t {
        const int64_t u = (t / B) * kPencil + w;
        return u < nu ? u : nu - 1;
      };
      auto row_in = [&](int64_t t, int64_t a) -> int64_t {
        const int64_t u = (t / B) * kPencil + w;
        const int64_t r = a + (t % B) * RPW + l;
        return (t * RPI < total && u < nu && r < (((a >> kUnitLog2) + 1) << kUnitLog2) && r < P.se) ? r : -1;
      };
      int64_t t = P.j;
      int64_t a0 = units[unit_of(t)];
      int64_t a1 = units[unit_of(t + g)];
      {
        const int64_t r = row_in(t, a0);
        ldk(r >= 0 ? r : a0, kc);
      }
      for (; t * RPI < total; t += g) {
        const int64_t a2 = units[unit_of(t + 2 * g)];
        const int64_t rn = row_in(t + g, a1);
        ldk(rn >= 0 ? rn : a1, kn);
        const int64_t r = row_in(t, a0);
        run(r, r >= 0);
#pragma unroll
        for (int j = 0; j < KL; ++j) kc[j] = kn[j];
        a0 = a1;
        a1 = a2;
      }
      return;
    }
    // banded: unit starts are loaded two tiles ahead, keys one tile ahead
    const int64_t total = row_seq_len(P, A.units);
    if (total <= 0) return;
    const int32_t* __restrict__ units = A.units + P.u0;
    const int64_t lastu = (total - 1) >> kUnitLog2;
    constexpr int64_t um = (int64_t(1) << kUnitLog2) - 1;
    auto unit_of = [&](int64_t p) -> int64_t { const int64_t u = p >> kUnitLog2; return u < lastu ? u : lastu; };
    // row at position p of a tile whose unit starts at a, or -1 (past the unit or segment end)
    auto row_in = [&](int64_t p, int64_t a) -> int64_t {
      const int64_t r = a + (p & um);
      return (p < total && r < (((a >> kUnitLog2) + 1) << kUnitLog2) && r < P.se) ? r : -1;
    };
    int64_t pos = (int64_t)P.j * RPI + threadIdx.x / B;
    int64_t a0 = units[unit_of(pos)];
    int64_t a1 = units[unit_of(pos + step)];
    {
      const int64_t r = row_in(pos, a0);
      ldk(r >= 0 ? r : a0, kc);
    }
    for (int64_t pos0 = (int64_t)P.j * RPI; pos0 < total; pos0 += step, pos += step) {
      const int64_t a2 = units[unit_of(pos + 2 * step)];
      const int64_t rn = row_in(pos + step, a1);
      ldk(rn >= 0 ? rn : a1, kn);
      const int64_t r = row_in(pos, a0);
      run(r, r >= 0);
#pragma unroll
      for (int j = 0; j < KL; ++j) kc[j] = kn[j];
      a0 = a1;
      a1 = a2;
    }
  }
}

// Sum of v over the B lanes of one row (adjacent lanes, B a power of two).
template <int B>
__device__ __forceinline__ double row_lanes_sum(double v) {
#pragma unroll
  for (int off = 1; off < B; off <<= 1) v += __shfl_xor(v, off);
  return v;
}

// Per-entry gradients of row r: for every entry j (column c, not padding),
// g = f * sum over the row's B lanes of conj(lam) u_c, accumulated as
// (Re g, -Im g) at gH[r*ldH + j] by the row's first lane.  Every lane of the
// row calls this (the lane sums are shuffles).  Slot j of the sliced layout is
// slot j of the row in the input neighbour list.
template <int B, int HOP, int K>
__device__ __forceinline__ void row_entry_grads(const DevMat& A, int64_t r, int b, double2 lam,
                                                const double2* __restrict__ u, double f, double* gH, int ldH) {
  const int S = 1 << A.S_log2;
  const int64_t sl = r >> A.S_log2;
  const int64_t p0 = K > 0 ? sl * ((int64_t)K << A.S_log2) : A.slice_ptr[sl];
  const int64_t e0 = p0 + (r & (S - 1));
  const int w = K > 0 ? K : (int)((A.slice_ptr[sl + 1] - p0) >> A.S_log2);
  for (int j = 0; j < w; ++j) {
    const int64_t e = e0 + (int64_t)j * S;
    int64_t cc;
    const bool ok = col_entry<HOP>(A, r, e, &cc);
    const double2 x = u[cc * B + b];
    double gr = lam.x * x.x + lam.y * x.y;   // conj(lam) x
    double gi = lam.x * x.y - lam.y * x.x;
    gr = row_lanes_sum<B>(gr);
    gi = row_lanes_sum<B>(gi);
    if (ok && b == 0) {
      double* p = gH + 2 * (r * (int64_t)ldH + j);
      p[0] += f * gr;
      p[1] -= f * gi;
    }
  }
}

// Sum (re, im) over the lanes of the workgroup that share column b = tid % B,
// in a fixed order, and store one partial per column.
template <int B>
__device__ __forceinline__ void block_reduce_store(double re, double im, double2* __restrict__ dst) {
  __shared__ double sh[2][kBlock / 64][B];
#pragma unroll
  for (int off = 32; off >= B; off >>= 1) {
    re += __shfl_xor(re, off);
    im += __shfl_xor(im, off);
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (lane < B) {
    sh[0][wave][lane] = re;
    sh[1][wave][lane] = im;
  }
  __syncthreads();
  if (threadIdx.x < B) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
      sr += sh[0][q][threadIdx.x];
      si += sh[1][q][threadIdx.x];
    }
    dst[threadIdx.x] = make_double2(sr, si);
  }
}

// ---------------------------------------------------------------------------
// compile-time dispatch: B x hopping mode x non-temporal x row width
// ---------------------------------------------------------------------------
template <typename F>
inline hipError_t dispatch_bh(int B, int hop_mode, F&& f) {
  auto on_b = [&](auto Bc) {
    if (hop_mode == HOP_UNIFORM) f(Bc, IC<HOP_UNIFORM>{});
    else if (hop_mode == HOP_REAL) f(Bc, IC<HOP_REAL>{});
    else if (hop_mode == HOP_COMPLEX) f(Bc, IC<HOP_COMPLEX>{});
    else f(Bc, IC<HOP_DICT>{});
  };
  switch (B) {
    case 1: on_b(IC<1>{}); break;
    case 2: on_b(IC<2>{}); break;
    case 4: on_b(IC<4>{}); break;
    case 8: on_b(IC<8>{}); break;
    case 16: on_b(IC<16>{}); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename F>
inline hipError_t dispatch_sparse(const DevMat& A, int hop_mode, int B, int nt, F&& f) {
  return dispatch_bh(B, hop_mode, [&](auto Bc, auto Hc) {
    auto on_k = [&](auto NTc) {
      switch (A.K) {
        case 3: f(Bc, Hc, IC<3>{}, NTc); break;
        case 4: f(Bc, Hc, IC<4>{}, NTc); break;
        case 6: f(Bc, Hc, IC<6>{}, NTc); break;
        case 8: f(Bc, Hc, IC<8>{}, NTc); break;
        default: f(Bc, Hc, IC<0>{}, NTc); break;
      }
    };
    if (nt) on_k(std::true_type{});
    else on_k(std::false_type{});
  });
}


}  // namespace dev
}  // namespace gpuqt
