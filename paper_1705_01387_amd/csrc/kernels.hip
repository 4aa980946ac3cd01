// HIP kernels for gfx950 (CDNA4): the sparse Chebyshev steps of the
// linear-scaling Kubo method and their helpers.
//
// Every sparse kernel streams the sliced-ELL Hamiltonian once per launch:
// one row (for B > 1, one (row, column) pair per lane with the B lanes of a
// row adjacent) per lane, slot-major entries so that a wavefront reading one
// slot of consecutive rows touches consecutive addresses, 16-byte loads of
// complex128 vector elements, FP64 throughout (no MFMA: a step moves about
// 20 bytes per FP64 multiply-add pair, far below the matrix-core balance).
//
// Schedule: G workgroups of 256 threads.  The hardware hands workgroups to
// the 8 XCDs round-robin, so physical workgroup p becomes logical workgroup
// (p % 8) * (G / 8) + p / 8; the logical workgroups of one XCD that work on
// one segment form a group owning a contiguous row range, and walk it in
// tiles of 256/B rows with stride "group size".  All workgroups resident on
// an XCD therefore sweep one compact window of rows together: a neighbour
// gather (e.g. one lattice plane away) finds the line its neighbours fetched
// moments ago in that XCD's L2 or in the last-level cache, instead of
// re-reading it from HBM.
//
// NT variants mark the once-read streams (indices, hoppings, position
// differences, on-site terms, v_{n-2}, phi_L) non-temporal so that they do
// not push the gathered vector out of the caches.
//
// Moment reductions are deterministic: wavefront butterfly, then a fixed
// order over the four wavefronts, one partial per workgroup and step, and a
// fixed-shape final reduction over workgroups.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <type_traits>

#include "bessel.h"
#include "internal.h"

#include "device_common.h"

namespace gpuqt {

using namespace dev;

namespace {

// ---------------------------------------------------------------------------
// Chebyshev moment step (Sections 3.2-3.3): v_n = 2 H~ v_{n-1} - v_{n-2}
// (v_1 = H~ v_0) and the workgroup's part of <phiL|v_n> (and <phiL|v_0>).
// ---------------------------------------------------------------------------
template <int B, int HOP, int K, bool NT>
__global__ __launch_bounds__(kBlock) void k_moment_step(DevMat A, StepIO io,
                                                        const double2* __restrict__ phiL,
                                                        double2* __restrict__ part_n,
                                                        double2* __restrict__ part_0) {
  const int lb = logical_block(A.G);
  const BlkPlan P = A.plan[lb];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const int b = threadIdx.x & (B - 1);
  const double2* __restrict__ x = io.x;
  const double2* __restrict__ w = io.w;
  double2* __restrict__ out = io.out;
  const bool first = io.first;
  // per-row operands that need no column index are loaded first (w is read
  // from x on the first step, where it is unused, to keep the load unconditional)
  const double2* __restrict__ wsrc = first ? x : w;
  double dr = 0.0, di = 0.0, zr = 0.0, zi = 0.0;
  for_rows_pf<B, HOP, K, NT>(A, P, [&](int64_t r, const int32_t* kc) {
    const int64_t idx = r * B + b;
    const double2 xr = x[idx];
    const double2 wv = ld2<NT>(wsrc + idx);
    double2 p = make_double2(0.0, 0.0);
    if (phiL) p = ld2<NT>(phiL + idx);   // plain recurrence step (no moment) when phiL is NULL
    double2 ha, hb, da;
    row_apply<B, HOP, K, NT, false, false, true>(A, r, b, hu, x, nullptr, xr, xr, ha, hb, da, kc);
    const double2 y = first ? ha : twice_minus(ha, wv);
    out[idx] = y;
    if (phiL) {
      cdot_acc(dr, di, p, y);
      if (first) cdot_acc(zr, zi, p, xr);
    }
  });
  if (!phiL) return;
  block_reduce_store<B>(dr, di, part_n + (int64_t)lb * B);
  if (first) {
    __syncthreads();
    block_reduce_store<B>(zr, zi, part_0 + (int64_t)lb * B);
  }
}

// ---------------------------------------------------------------------------
// Moment step for a Hermitian moment set (phiL = phiR = v_0): the same
// recurrence, but the moments come from the product identities
//   T_{2k} = 2 T_k T_k - T_0,   T_{2k-1} = 2 T_k T_{k-1} - T_1,
// so step k yields the raw dots <v_k|v_{k-1}> (row 2k-1) and <v_k|v_k>
// (row 2k); the first step also <v_0|v_0> (row 0) and <v_0|v_1> (row 1).
// k_reduce turns raw rows n >= 2 into 2 raw_n - mu_{n mod 2}.  Half the
// steps of the plain recurrence, and no phi_L stream.
// ---------------------------------------------------------------------------
template <int B, int HOP, int K, bool NT>
__global__ __launch_bounds__(kBlock) void k_moment_step_sym(DevMat A, StepIO io,
                                                            double2* __restrict__ part_a,
                                                            double2* __restrict__ part_b,
                                                            double2* __restrict__ part_c) {
  const int lb = logical_block(A.G);
  const BlkPlan P = A.plan[lb];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const int b = threadIdx.x & (B - 1);
  const double2* __restrict__ x = io.x;
  const double2* __restrict__ w = io.w;
  double2* __restrict__ out = io.out;
  const bool first = io.first;
  // first: a = <v0|v0>, b = <v0|v1>, c = <v1|v1>;  else: a = <vk|vk-1>, c = <vk|vk>
  const double2* __restrict__ wsrc = first ? x : w;   // w unused on the first step
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0, cr = 0.0, ci = 0.0;
  for_rows_pf<B, HOP, K, NT>(A, P, [&](int64_t r, const int32_t* kc) {
    const int64_t idx = r * B + b;
    const double2 xr = x[idx];
    double2 ha, hb, da;
    row_apply<B, HOP, K, NT, false, false, true>(A, r, b, hu, x, nullptr, xr, xr, ha, hb, da, kc);
    const double2 wv = ld2<NT>(wsrc + idx);
    const double2 y = first ? ha : twice_minus(ha, wv);
    out[idx] = y;
    if (first) {
      cdot_acc(ar, ai, xr, xr);
      cdot_acc(br, bi, xr, y);
    } else {
      cdot_acc(ar, ai, y, xr);
    }
    cdot_acc(cr, ci, y, y);
  });
  block_reduce_store<B>(ar, ai, part_a + (int64_t)lb * B);
  __syncthreads();
  block_reduce_store<B>(cr, ci, part_c + (int64_t)lb * B);
  if (first) {
    __syncthreads();
    block_reduce_store<B>(br, bi, part_b + (int64_t)lb * B);
  }
}

// ---------------------------------------------------------------------------
// The Hermitian moment step of k_moment_step_sym on a periodic box (every row
// x + Lx (y + Ly z) with the six neighbours one step away in x, y and z, one
// uniform hopping; detect_box), for blocks of B >= 2 vectors.  The gathers of
// the general kernel fetch every element of x through the L1 five times per
// step (as the row's own element and as the neighbour one line and one plane
// away on either side).  Here a workgroup owns a TX x TY column of the box and
// a run of zc planes and marches through them: each lane keeps its elements of
// planes z - 1, z and z + 1 in registers (the z neighbours), plane z of the
// tile and its one-row halo go to LDS (the x and y neighbours), so x is read
// about (1 + halo) times instead of five, and the neighbour indices are not
// read at all.  Everything plane z + 1 needs (x of plane z + 2, the halo of
// z + 1, w and the diagonal) is loaded while plane z is computed; one barrier
// per plane (double-buffered LDS).  Addresses are a plane base, uniform over
// the workgroup, plus a 32-bit byte offset per lane that is fixed for the run
// (a plane of the block must span less than 4 GiB; box_fits).  Positions of a
// tile past the box edge hold the wrapped rows (so the edge rows' periodic
// neighbours are in place) and produce no output.  Work items (column, run of
// planes) go round the G workgroups, each writing one partial like the
// general kernel; the column index runs fastest, so the workgroups of one XCD
// (consecutive logical blocks) hold a band of neighbouring columns at the same
// run and march through z together, and the halo rows they read from each
// other are hits in that XCD's L2.
// ---------------------------------------------------------------------------

// Which elements of a TX x TY box tile (plus its one-cell halo without the
// corners) this thread handles, their LDS slots, and per work item their byte
// offsets inside a plane of a block of B vectors and of the diagonal.
template <int B, int TX, int TY>
struct BoxTile {
  static constexpr int PX = TX + 2, PY = TY + 2, PE = PX * PY * B;   // staged elements per plane
  static constexpr int OE = TX * TY * B;                              // own elements per plane
  static_assert(OE % kBlock == 0, "a tile plane must give every thread the same count");
  static constexpr int OPT = OE / kBlock;
  static constexpr int HE = (2 * TX + 2 * TY) * B;                    // halo elements
  static constexpr int HPT = (HE + kBlock - 1) / kBlock;
  // hval: the lane's halo element exists (HE is not always a multiple of kBlock); the
  // other lanes load the element of lane e mod HE instead and do not stage it, so that
  // every lane issues the same loads (a load under a lane test would make the compiler
  // wait for all loads in flight, prefetches included, where the branches join)
  int oslot[OPT], olx[OPT], oly[OPT], hslot[HPT], hpx[HPT], hpy[HPT];
  bool hval[HPT], oval[OPT];
  uint32_t oo[OPT], od[OPT], ho[HPT];   // own element, own diagonal, halo element

  __device__ __forceinline__ explicit BoxTile(int b) {
#pragma unroll
    for (int i = 0; i < OPT; ++i) {
      const int p = (threadIdx.x + i * kBlock) / B;
      olx[i] = p % TX;
      oly[i] = p / TX;
      oslot[i] = ((oly[i] + 1) * PX + olx[i] + 1) * B + b;
    }
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
      const int e = threadIdx.x + j * kBlock;
      const int q = (e % HE) / B;
      hval[j] = e < HE;
      int px = 0, py = 0;
      if (q < TX) {
        px = q + 1;
      } else if (q < 2 * TX) {
        px = q - TX + 1;
        py = PY - 1;
      } else if (q < 2 * TX + TY) {
        py = q - 2 * TX + 1;
      } else {
        px = PX - 1;
        py = q - 2 * TX - TY + 1;
      }
      hpx[j] = px;
      hpy[j] = py;
      hslot[j] = (py * PX + px) * B + b;
    }
  }

  // the tile whose first cell is (x0, y0)
  __device__ __forceinline__ void place(int x0, int y0, int Lx, int Ly, int b) {
    auto wrap = [](int v, int L) { return ((v % L) + L) % L; };
#pragma unroll
    for (int i = 0; i < OPT; ++i) {
      const int X = x0 + olx[i], Y = y0 + oly[i];
      oval[i] = X < Lx && Y < Ly;
      const uint32_t row = (uint32_t)wrap(Y, Ly) * (uint32_t)Lx + (uint32_t)wrap(X, Lx);
      oo[i] = (row * B + b) * (uint32_t)sizeof(double2);
      od[i] = row * (uint32_t)sizeof(double);
    }
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
      const uint32_t row = (uint32_t)wrap(y0 + hpy[j] - 1, Ly) * (uint32_t)Lx + (uint32_t)wrap(x0 + hpx[j] - 1, Lx);
      ho[j] = (row * B + b) * (uint32_t)sizeof(double2);
    }
  }
};

// The streams a box kernel reads or writes once per step (everything but the
// staged chains) carry the non-temporal hint, so that they do not push the
// staged planes, which neighbouring tiles read again as halo, out of the L2
// (cubic 200^3: the B = 4 Hermitian step 318 -> 308 us, the MSD term
// 1080 -> 1036 us, B = 16 1288 -> 1217 us).
constexpr bool kBoxNtLoad = true, kBoxNtStore = true;

template <bool NT = false>
__device__ __forceinline__ double2 box_ld(const char* base, uint32_t off) {
  return ld2<NT>(reinterpret_cast<const double2*>(base + off));
}
__device__ __forceinline__ void box_st(char* base, uint32_t off, double2 v) {
  if constexpr (kBoxNtStore) {
    const d2v t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<d2v*>(base + off));
  } else {
    *reinterpret_cast<double2*>(base + off) = v;
  }
}
__device__ __forceinline__ double box_ldd(const char* base, uint32_t off) {
  if constexpr (kBoxNtLoad) return __builtin_nontemporal_load(reinterpret_cast<const double*>(base + off));
  return *reinterpret_cast<const double*>(base + off);
}

template <int B, int TX, int TY, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_moment_step_sym_box(DevMat A, StepIO io, int zc,
                                                                double2* __restrict__ part_a,
                                                                double2* __restrict__ part_b,
                                                                double2* __restrict__ part_c) {
  using T = BoxTile<B, TX, TY>;
  constexpr int OPT = T::OPT, HPT = T::HPT, PX = T::PX;
  __shared__ double2 lds[2][T::PE];
  const int lb = logical_block(A.G);
  const int Lx = A.box[0], Ly = A.box[1], Lz = A.box[2];
  const int txn = (Lx + TX - 1) / TX, tyn = (Ly + TY - 1) / TY, zn = (Lz + zc - 1) / zc;
  const int64_t cols = (int64_t)txn * tyn, items = cols * zn;
  const double hu = A.seg_hop[0];
  const int b = threadIdx.x & (B - 1);
  const char* xs = reinterpret_cast<const char*>(io.x);
  const char* ws = reinterpret_cast<const char*>(io.w);   // not read on the first step
  char* os = reinterpret_cast<char*>(io.out);
  const char* ds = reinterpret_cast<const char*>(A.diag);
  const int64_t vplane = (int64_t)Lx * Ly * B * (int64_t)sizeof(double2);
  const int64_t dplane = (int64_t)Lx * Ly * (int64_t)sizeof(double);
  auto zw = [Lz](int z) { return z < 0 ? z + Lz : (z >= Lz ? z - Lz : z); };   // z in [-1, Lz + 1]
  T t(b);
  // first: a = <v0|v0>, b = <v0|v1>, c = <v1|v1>;  else: a = <vk|vk-1>, c = <vk|vk>
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0, cr = 0.0, ci = 0.0;
  for (int64_t it = lb; it < items; it += A.G) {
    const int tz = (int)(it / cols);
    const int64_t txy = it % cols;
    const int z0 = tz * zc, z1 = min(z0 + zc, Lz);
    t.place((int)(txy % txn) * TX, (int)(txy / txn) * TY, Lx, Ly, b);
    // x of planes z - 1, z, z + 1 and the one loaded for z + 2 rotate through x0..x3; w,
    // the diagonal and the halo of planes z and z + 1 through (w0, w1), (d0, d1), (h0, h1).
    // The loop below is unrolled four planes deep so that the rotation is a renaming: a
    // register copy of a load in flight would wait for it.
    double2 x0[OPT], x1[OPT], x2[OPT], x3[OPT], w0[OPT], w1[OPT], h0[HPT], h1[HPT];
    double d0[OPT], d1[OPT];
    {
      const char* xa = xs + zw(z0 - 1) * vplane;
      const char* xb = xs + z0 * vplane;
      const char* xd = xs + zw(z0 + 1) * vplane;
#pragma unroll
      for (int i = 0; i < OPT; ++i) {
        x0[i] = box_ld(xa, t.oo[i]);
        x1[i] = box_ld(xb, t.oo[i]);
        x2[i] = box_ld(xd, t.oo[i]);
        w0[i] = FIRST ? make_double2(0.0, 0.0) : box_ld<kBoxNtLoad>(ws + z0 * vplane, t.oo[i]);
        d0[i] = box_ldd(ds + z0 * dplane, t.od[i]);
      }
#pragma unroll
      for (int j = 0; j < HPT; ++j) h0[j] = box_ld(xb, t.ho[j]);
    }
    // plane z, staged in LDS buffer BF: first the loads for plane z + 1 (on the last plane
    // of the run they read the planes after it, wrapped into the box, and go unused: the
    // same loads on every plane keep the wait for plane z's operands from waiting for
    // these too), then the stencil
    auto plane = [&](int z, auto BF, double2(&xm)[OPT], double2(&xc)[OPT], double2(&xp)[OPT],
                     double2(&xq)[OPT], double2(&wc)[OPT], double2(&wn)[OPT], double(&dc)[OPT],
                     double(&dn)[OPT], double2(&hc)[HPT], double2(&hn)[HPT]) {
      constexpr int bf = decltype(BF)::value;
      const int z1n = zw(z + 1);
      const char* xq_ = xs + zw(z + 2) * vplane;
      const char* xn_ = xs + z1n * vplane;
#pragma unroll
      for (int i = 0; i < OPT; ++i) {
        xq[i] = box_ld(xq_, t.oo[i]);
        if (!FIRST) wn[i] = box_ld<kBoxNtLoad>(ws + z1n * vplane, t.oo[i]);
        dn[i] = box_ldd(ds + z1n * dplane, t.od[i]);
      }
#pragma unroll
      for (int j = 0; j < HPT; ++j) hn[j] = box_ld(xn_, t.ho[j]);
#pragma unroll
      for (int i = 0; i < OPT; ++i) lds[bf][t.oslot[i]] = xc[i];
#pragma unroll
      for (int j = 0; j < HPT; ++j)
        if (t.hval[j]) lds[bf][t.hslot[j]] = hc[j];
      __syncthreads();
      char* oz = os + z * vplane;
#pragma unroll
      for (int i = 0; i < OPT; ++i) {
        if (t.oval[i]) {
          const int c = t.oslot[i];
          double2 sn = cadd(lds[bf][c + B], lds[bf][c - B]);
          sn = cadd(sn, lds[bf][c + PX * B]);
          sn = cadd(sn, lds[bf][c - PX * B]);
          sn = cadd(sn, xp[i]);
          sn = cadd(sn, xm[i]);
          const double2 xr = xc[i];
          const double2 h = make_double2(fma(dc[i], xr.x, hu * sn.x), fma(dc[i], xr.y, hu * sn.y));
          const double2 y = FIRST ? h : twice_minus(h, wc[i]);
          box_st(oz, t.oo[i], y);
          if (FIRST) {
            cdot_acc(ar, ai, xr, xr);
            cdot_acc(br, bi, xr, y);
          } else {
            cdot_acc(ar, ai, y, xr);
          }
          cdot_acc(cr, ci, y, y);
        }
      }
    };
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    for (int z = z0; z < z1; z += 4) {
      plane(z, S0{}, x0, x1, x2, x3, w0, w1, d0, d1, h0, h1);
      if (z + 1 >= z1) break;
      plane(z + 1, S1{}, x1, x2, x3, x0, w1, w0, d1, d0, h1, h0);
      if (z + 2 >= z1) break;
      plane(z + 2, S0{}, x2, x3, x0, x1, w0, w1, d0, d1, h0, h1);
      if (z + 3 >= z1) break;
      plane(z + 3, S1{}, x3, x0, x1, x2, w1, w0, d1, d0, h1, h0);
    }
    __syncthreads();   // the next item stages into buffer 0 again
  }
  block_reduce_store<B>(ar, ai, part_a + (int64_t)lb * B);
  __syncthreads();
  block_reduce_store<B>(cr, ci, part_c + (int64_t)lb * B);
  if (FIRST) {
    __syncthreads();
    block_reduce_store<B>(br, bi, part_b + (int64_t)lb * B);
  }
}

// ---------------------------------------------------------------------------
// The Hermitian step of k_moment_step_sym on segments that are each a periodic
// Lx x Ly square (rows off_s + x + Lx y, four neighbours, one uniform hopping per
// segment; detect_sheets), for blocks of B >= 2 vectors: the two-dimensional form
// of k_moment_step_sym_box.  A workgroup holds a strip of TX = 256 / B cells of one
// row (a lane per cell and vector) and marches along y: rows y - 1, y and y + 1 of
// the strip stay in registers (the y neighbours), row y and its two halo cells go
// to LDS (the x neighbours).  The workgroups of segment s (sheet_blk0: the plan's
// workgroups split over the segments by their work, so that the segments finish
// together) take its work items (strip, run of sheet_zc rows), strip index
// fastest, so the workgroups of
// one XCD hold neighbouring strips of the same rows.  Loads for row y + 1 are
// issued unconditionally while row y is computed and the march is unrolled four
// rows deep, as in the box kernel.
// ---------------------------------------------------------------------------
template <int B, int OPT, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_moment_step_sym_sheet(DevMat A, StepIO io,
                                                                  double2* __restrict__ part_a,
                                                                  double2* __restrict__ part_b,
                                                                  double2* __restrict__ part_c) {
  constexpr int TL = kBlock / B;               // cells per lane row of the strip
  constexpr int TX = OPT * TL, PX = TX + 2;    // cells per strip: OPT per lane
  __shared__ double2 lds[2][PX * B];
  const int lb = logical_block(A.G);
  // this workgroup's segment in the kernel's own split (sheet_blk0: by work, not rows)
  int sg = 0;
  for (int hi = A.sheet_nseg - 1; sg < hi;) {
    const int mid = (sg + hi + 1) >> 1;
    if (A.sheet_blk0[mid] <= lb) sg = mid;
    else hi = mid - 1;
  }
  const int Lx = A.sheet[2 * sg], Ly = A.sheet[2 * sg + 1];
  const int zc = A.sheet_zc[sg];
  const int w0 = A.sheet_blk0[sg], nw = A.sheet_blk0[sg + 1] - w0;
  const int64_t off = A.sheet_off[sg];
  const int cols = (Lx + TX - 1) / TX, zn = (Ly + zc - 1) / zc;
  const int64_t items = (int64_t)cols * zn;
  const double hu = A.seg_hop[sg];
  const int b = threadIdx.x & (B - 1);
  const int cx = threadIdx.x / B;                       // first cell of this lane in the strip
  const char* xs = reinterpret_cast<const char*>(io.x + off * B);
  const char* ws = reinterpret_cast<const char*>((FIRST ? io.x : io.w) + off * B);   // not read when FIRST
  char* os = reinterpret_cast<char*>(io.out + off * B);
  const char* ds = reinterpret_cast<const char*>(A.diag + off);
  const int64_t vrow = (int64_t)Lx * B * (int64_t)sizeof(double2), drow = (int64_t)Lx * (int64_t)sizeof(double);
  auto zw = [Ly](int y) { return y < 0 ? y + Ly : (y >= Ly ? y - Ly : y); };   // y in [-1, Ly + 1]
  auto wrap = [](int v, int L) { return ((v % L) + L) % L; };
  // halo: lanes 0 .. B - 1 stage the cell left of the strip, B .. 2B - 1 the one right of
  // it; the other lanes load lane (threadIdx.x mod 2B)'s element and do not stage it
  const bool hval = threadIdx.x < 2 * B;
  const bool hright = (threadIdx.x % (2 * B)) >= B;
  const int hslot = (hright ? PX - 1 : 0) * B + b;
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0, cr = 0.0, ci = 0.0;
  for (int64_t it = lb - w0; it < items; it += nw) {
    const int tz = (int)(it / cols), strip = (int)(it % cols);
    const int x0 = strip * TX;
    const int y0 = tz * zc, y1 = min(y0 + zc, Ly);
    bool oval[OPT];
    uint32_t oo[OPT], od[OPT];
#pragma unroll
    for (int i = 0; i < OPT; ++i) {
      const int X = x0 + cx + i * TL;
      oval[i] = X < Lx;
      const uint32_t xo = (uint32_t)wrap(X, Lx);
      oo[i] = (xo * B + b) * (uint32_t)sizeof(double2);
      od[i] = xo * (uint32_t)sizeof(double);
    }
    const uint32_t ho = ((uint32_t)wrap(hright ? x0 + TX : x0 - 1, Lx) * B + b) * (uint32_t)sizeof(double2);
    // x of rows y - 1, y, y + 1 and the one loaded for y + 2 rotate through q0..q3; w, the
    // diagonal and the halo of rows y and y + 1 through pairs (unrolled four rows deep)
    double2 q0[OPT], q1[OPT], q2[OPT], q3[OPT], wa[OPT], wb[OPT], h0, h1;
    double d0[OPT], d1[OPT];
#pragma unroll
    for (int i = 0; i < OPT; ++i) {
      q0[i] = box_ld(xs + zw(y0 - 1) * vrow, oo[i]);
      q1[i] = box_ld(xs + y0 * vrow, oo[i]);
      q2[i] = box_ld(xs + zw(y0 + 1) * vrow, oo[i]);
      wa[i] = FIRST ? make_double2(0.0, 0.0) : box_ld<kBoxNtLoad>(ws + y0 * vrow, oo[i]);
      wb[i] = make_double2(0.0, 0.0);
      d0[i] = box_ldd(ds + y0 * drow, od[i]);
    }
    h0 = box_ld(xs + y0 * vrow, ho);
    auto row = [&](int y, auto BF, double2(&xm)[OPT], double2(&xc)[OPT], double2(&xp)[OPT], double2(&xq)[OPT],
                   double2(&wc)[OPT], double2(&wn)[OPT], double(&dc)[OPT], double(&dn)[OPT], double2& hc,
                   double2& hn) {
      constexpr int bf = decltype(BF)::value;
      const int y1n = zw(y + 1);
#pragma unroll
      for (int i = 0; i < OPT; ++i) {
        xq[i] = box_ld(xs + zw(y + 2) * vrow, oo[i]);
        if (!FIRST) wn[i] = box_ld<kBoxNtLoad>(ws + y1n * vrow, oo[i]);
        dn[i] = box_ldd(ds + y1n * drow, od[i]);
      }
      hn = box_ld(xs + y1n * vrow, ho);
#pragma unroll
      for (int i = 0; i < OPT; ++i) lds[bf][(cx + i * TL + 1) * B + b] = xc[i];
      if (hval) lds[bf][hslot] = hc;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < OPT; ++i) {
        if (oval[i]) {
          const int c = (cx + i * TL + 1) * B + b;
          double2 sn = cadd(lds[bf][c + B], lds[bf][c - B]);
          sn = cadd(sn, xp[i]);
          sn = cadd(sn, xm[i]);
          const double2 xr = xc[i];
          const double2 h = make_double2(fma(dc[i], xr.x, hu * sn.x), fma(dc[i], xr.y, hu * sn.y));
          const double2 yv = FIRST ? h : twice_minus(h, wc[i]);
          box_st(os + y * vrow, oo[i], yv);
          if (FIRST) {
            cdot_acc(ar, ai, xr, xr);
            cdot_acc(br, bi, xr, yv);
          } else {
            cdot_acc(ar, ai, yv, xr);
          }
          cdot_acc(cr, ci, yv, yv);
        }
      }
    };
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    for (int y = y0; y < y1; y += 4) {
      row(y, S0{}, q0, q1, q2, q3, wa, wb, d0, d1, h0, h1);
      if (y + 1 >= y1) break;
      row(y + 1, S1{}, q1, q2, q3, q0, wb, wa, d1, d0, h1, h0);
      if (y + 2 >= y1) break;
      row(y + 2, S0{}, q2, q3, q0, q1, wa, wb, d0, d1, h0, h1);
      if (y + 3 >= y1) break;
      row(y + 3, S1{}, q3, q0, q1, q2, wb, wa, d1, d0, h1, h0);
    }
    __syncthreads();   // the next item stages into buffer 0 again
  }
  block_reduce_store<B>(ar, ai, part_a + (int64_t)lb * B);
  __syncthreads();
  block_reduce_store<B>(cr, ci, part_c + (int64_t)lb * B);
  if (FIRST) {
    __syncthreads();
    block_reduce_store<B>(br, bi, part_b + (int64_t)lb * B);
  }
}

// ---------------------------------------------------------------------------
// Moment step for <a|T_n|b> with a != b: both chains a_k = T_k a, b_k = T_k b
// advance in one launch (one matrix read, the two gathers share the indices)
// and the identities give
//   <a|T_{2k}|b> = 2 <a_k|b_k> - <a|b>,  <a|T_{2k-1}|b> = 2 <a_k|b_{k-1}> - <a|T_1 b>,
// so step k yields <a_k|b_{k-1}> (row 2k-1) and <a_k|b_k> (row 2k); the first
// step also <a|b> (row 0) and <a|b_1> (row 1).
// ---------------------------------------------------------------------------
template <int B, int HOP, int K, bool NT>
__global__ __launch_bounds__(kBlock) void k_moment_step_pair(DevMat A, ChainIO io,
                                                             double2* __restrict__ part_a,
                                                             double2* __restrict__ part_b,
                                                             double2* __restrict__ part_c) {
  const int lb = logical_block(A.G);
  const BlkPlan P = A.plan[lb];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const int b = threadIdx.x & (B - 1);
  const bool first = io.first;
  const double2* __restrict__ wa = first ? io.xa : io.wa;   // unused on the first step
  const double2* __restrict__ wb = first ? io.xb : io.wb;
  double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0, cr = 0.0, ci = 0.0;
  for_rows_pf<B, HOP, K, NT>(A, P, [&](int64_t r, const int32_t* kc) {
    const int64_t idx = r * B + b;
    const double2 xa = io.xa[idx];
    const double2 xb = io.xb[idx];
    const double2 wav = ld2<NT>(wa + idx);
    const double2 wbv = ld2<NT>(wb + idx);
    double2 ha, hb, da;
    row_apply<B, HOP, K, NT, true, false, true>(A, r, b, hu, io.xa, io.xb, xa, xb, ha, hb, da, kc);
    const double2 ya = first ? ha : twice_minus(ha, wav);
    const double2 yb = first ? hb : twice_minus(hb, wbv);
    io.oa[idx] = ya;
    io.ob[idx] = yb;
    if (first) {
      cdot_acc(ar, ai, xa, xb);
      cdot_acc(br, bi, xa, yb);
    } else {
      cdot_acc(ar, ai, ya, xb);
    }
    cdot_acc(cr, ci, ya, yb);
  });
  block_reduce_store<B>(ar, ai, part_a + (int64_t)lb * B);
  __syncthreads();
  block_reduce_store<B>(cr, ci, part_c + (int64_t)lb * B);
  if (first) {
    __syncthreads();
    block_reduce_store<B>(br, bi, part_b + (int64_t)lb * B);
  }
}

// ---------------------------------------------------------------------------
// One term m of U(dt) psi = sum_m c_m T_m(H~) psi (Section 3.2):
// a_m by the recurrence, acc += c_m a_m; c_m = J[seg][m] * phase_m with the
// table holding (2 - delta_m0) J_m(DeltaE_seg |dt|).
// ---------------------------------------------------------------------------
template <int B, int HOP, int K, bool NT>
__global__ __launch_bounds__(kBlock) void k_evolve_term(DevMat A, StepIO io, double2* __restrict__ acc,
                                                        const double* __restrict__ Jtab, int ldJ,
                                                        int m, double2 ph_m, double2 ph_0) {
  const BlkPlan P = A.plan[logical_block(A.G)];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const double2 cm = cscale(Jtab[(int64_t)P.seg * ldJ + m], ph_m);
  const double2 c0 = cscale(Jtab[(int64_t)P.seg * ldJ], ph_0);
  const int b = threadIdx.x & (B - 1);
  const double2* __restrict__ x = io.x;
  const double2* __restrict__ w = io.w;
  double2* __restrict__ out = io.out;
  const bool first = io.first;
  // w and acc are unused on the first step: read x there instead, so that the
  // loads stay unconditional and ahead of the gathers
  const double2* __restrict__ wsrc = first ? x : w;
  const double2* __restrict__ asrc = first ? x : acc;
  for_rows_pf<B, HOP, K, NT>(A, P, [&](int64_t r, const int32_t* kc) {
    const int64_t idx = r * B + b;
    const double2 xr = x[idx];
    const double2 wv = ld2<NT>(wsrc + idx);
    const double2 av = ld2<NT>(asrc + idx);
    double2 ha, hb, da;
    row_apply<B, HOP, K, NT, false, false, true>(A, r, b, hu, x, nullptr, xr, xr, ha, hb, da, kc);
    if (first) {
      out[idx] = ha;
      acc[idx] = cadd(cmul(c0, xr), cmul(cm, ha));
    } else {
      const double2 y = twice_minus(ha, wv);
      out[idx] = y;
      acc[idx] = cadd(av, cmul(cm, y));
    }
  });
}

// ---------------------------------------------------------------------------
// One term m of U(dt) applied to two vectors at once (both VAC states advance
// with the same U(-dt), Section 3.3): chains a_m = T_m psi_a, b_m = T_m psi_b
// share the matrix read and the gather indices; acc_a += c_m a_m,
// acc_b += c_m b_m.
// ---------------------------------------------------------------------------
template <int B, int HOP, int K, bool NT>
__global__ __launch_bounds__(kBlock) void k_evolve_pair_term(DevMat A, ChainIO io, double2* __restrict__ acc_a,
                                                             double2* __restrict__ acc_b,
                                                             const double* __restrict__ Jtab, int ldJ, int m,
                                                             double2 ph_m, double2 ph_0) {
  const BlkPlan P = A.plan[logical_block(A.G)];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const double2 cm = cscale(Jtab[(int64_t)P.seg * ldJ + m], ph_m);
  const double2 c0 = cscale(Jtab[(int64_t)P.seg * ldJ], ph_0);
  const int b = threadIdx.x & (B - 1);
  const bool first = io.first;
  // the w and acc operands are unused on the first step (read x there instead)
  const double2* __restrict__ wa = first ? io.xa : io.wa;
  const double2* __restrict__ wb = first ? io.xb : io.wb;
  const double2* __restrict__ sa = first ? io.xa : acc_a;
  const double2* __restrict__ sb = first ? io.xb : acc_b;
  for_rows_pf<B, HOP, K, NT>(A, P, [&](int64_t r, const int32_t* kc) {
    const int64_t idx = r * B + b;
    const double2 xa = io.xa[idx];
    const double2 xb = io.xb[idx];
    const double2 wav = ld2<NT>(wa + idx);
    const double2 wbv = ld2<NT>(wb + idx);
    const double2 aav = ld2<NT>(sa + idx);
    const double2 abv = ld2<NT>(sb + idx);
    double2 ha, hb, da;
    row_apply<B, HOP, K, NT, true, false, true>(A, r, b, hu, io.xa, io.xb, xa, xb, ha, hb, da, kc);
    if (first) {
      io.oa[idx] = ha;
      io.ob[idx] = hb;
      acc_a[idx] = cadd(cmul(c0, xa), cmul(cm, ha));
      acc_b[idx] = cadd(cmul(c0, xb), cmul(cm, hb));
    } else {
      const double2 ya = twice_minus(ha, wav);
      const double2 yb = twice_minus(hb, wbv);
      io.oa[idx] = ya;
      io.ob[idx] = yb;
      acc_a[idx] = cadd(aav, cmul(cm, ya));
      acc_b[idx] = cadd(abv, cmul(cm, yb));
    }
  });
}

// ---------------------------------------------------------------------------
// One term m of the fused evolution + commutator series (Section 3.2):
//   a_m = T_m psi:                a_1 = H~ a_0,  a_m = 2 H~ a_{m-1} - a_{m-2}
//   b_m = [X,T_m] psi + T_m chi:  b_0 = chi, b_1 = [X,H~] a_0 + H~ b_0,
//                                 b_m = 2 [X,H~] a_{m-1} + 2 H~ b_{m-1} - b_{m-2}
// (the sum of the paper's [X,T_m] recurrence and the T_m recurrence applied to
// chi); acc_a += c_m a_m, acc_b += c_m b_m.  [X,H~]_rj = -dx_rj H~_rj.
// ---------------------------------------------------------------------------
template <int B, int HOP, int K, bool NT>
__global__ __launch_bounds__(kBlock) void k_msd_term(DevMat A, ChainIO io, double2* __restrict__ acc_a,
                                                     double2* __restrict__ acc_b,
                                                     const double* __restrict__ Jtab, int ldJ, int m,
                                                     double2 ph_m, double2 ph_0) {
  const BlkPlan P = A.plan[logical_block(A.G)];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const double2 cm = cscale(Jtab[(int64_t)P.seg * ldJ + m], ph_m);
  const double2 c0 = cscale(Jtab[(int64_t)P.seg * ldJ], ph_0);
  const int b = threadIdx.x & (B - 1);
  const bool first = io.first;
  // the w and acc operands are unused on the first step (read x there instead)
  const double2* __restrict__ wa = first ? io.xa : io.wa;
  const double2* __restrict__ wb = first ? io.xb : io.wb;
  const double2* __restrict__ sa = first ? io.xa : acc_a;
  const double2* __restrict__ sb = first ? io.xb : acc_b;
  for_rows_pf<B, HOP, K, NT>(A, P, [&](int64_t r, const int32_t* kc) {
    const int64_t idx = r * B + b;
    const double2 xa = io.xa[idx];
    const double2 xb = io.xb[idx];
    const double2 wav = ld2<NT>(wa + idx);
    const double2 wbv = ld2<NT>(wb + idx);
    const double2 aav = ld2<NT>(sa + idx);
    const double2 abv = ld2<NT>(sb + idx);
    double2 ha, hb, da;
    row_apply<B, HOP, K, NT, true, true, true>(A, r, b, hu, io.xa, io.xb, xa, xb, ha, hb, da, kc);
    const double2 g = make_double2(hb.x - da.x, hb.y - da.y);   // [X,H~] a + H~ b
    if (first) {
      io.oa[idx] = ha;
      io.ob[idx] = g;
      acc_a[idx] = cadd(cmul(c0, xa), cmul(cm, ha));
      acc_b[idx] = cadd(cmul(c0, xb), cmul(cm, g));
    } else {
      const double2 ya = twice_minus(ha, wav);
      const double2 yb = twice_minus(g, wbv);
      io.oa[idx] = ya;
      io.ob[idx] = yb;
      acc_a[idx] = cadd(aav, cmul(cm, ya));
      acc_b[idx] = cadd(abv, cmul(cm, yb));
    }
  });
}

// ---------------------------------------------------------------------------
// Velocity V x (i sum dx H x) or [X,H] x (-sum dx H x), unscaled H
// (Section 4.2).  Stored values are H~ = H / DeltaE_seg, so multiply back.
// ---------------------------------------------------------------------------
template <int B, int HOP>
__global__ __launch_bounds__(kBlock) void k_commutator(DevMat A, int which, const double2* __restrict__ x,
                                                       double2* __restrict__ out) {
  const BlkPlan P = A.plan[logical_block(A.G)];
  const double hu = (HOP == HOP_UNIFORM) ? A.seg_hop[P.seg] : 0.0;
  const double e = A.seg_dE[P.seg];
  const int b = threadIdx.x & (B - 1);
  for_rows<B>(A, P, [&](int64_t r) {
    double2 ha, hb, da;
    const double2 z = make_double2(0.0, 0.0);   // no diagonal term: own element unused
    row_apply<B, HOP, 0, false, false, true, false>(A, r, b, hu, x, nullptr, z, z, ha, hb, da);
    const int64_t idx = r * B + b;
    double2 y;
    if ((which & 1) == GPUQT_VELOCITY) {
      y = make_double2(-e * da.y, e * da.x);   // i * e * da
    } else {
      y = make_double2(-e * da.x, -e * da.y);
    }
    out[idx] = (which & kAccumulate) ? cadd(out[idx], y) : y;
  });
}

// out = J_0(seg) * in, or zero when in is NULL.
template <int B>
__global__ __launch_bounds__(kBlock) void k_scale(DevMat A, const double2* __restrict__ in,
                                                  double2* __restrict__ out,
                                                  const double* __restrict__ Jtab, int ldJ) {
  const BlkPlan P = A.plan[logical_block(A.G)];
  const double j0 = Jtab ? Jtab[(int64_t)P.seg * ldJ] : 0.0;
  const int b = threadIdx.x & (B - 1);
  for_rows<B>(A, P, [&](int64_t r) {
    const int64_t idx = r * B + b;
    out[idx] = in ? cscale(j0, in[idx]) : make_double2(0.0, 0.0);
  });
}

// out = exp(i theta) with theta = 2 pi frac(0.618... idx + 0.414... b): a
// deterministic unit-modulus test vector (used only to time kernel variants).
template <int B>
__global__ __launch_bounds__(kBlock) void k_fill_phase(DevMat A, double2* __restrict__ out) {
  const BlkPlan P = A.plan[logical_block(A.G)];
  const int b = threadIdx.x & (B - 1);
  for_rows<B>(A, P, [&](int64_t r) {
    const double t = (double)r * 0.6180339887498949 + (double)b * 0.4142135623730951;
    double s, c;
    sincospi(2.0 * (t - floor(t)), &s, &c);
    out[r * B + b] = make_double2(c, s);
  });
}

__global__ void k_bessel_table(const double* __restrict__ seg_dE, int n_seg, double abs_dt, int Np,
                               int ldJ, double* __restrict__ J) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_seg) return;
  double* row = J + (int64_t)s * ldJ;
  bessel_miller(seg_dE[s] * abs_dt, Np, row);
  for (int m = 1; m < Np; ++m) row[m] *= 2.0;
}

// Sum of one partial row over the segment's workgroups, fixed order.
__device__ __forceinline__ double2 reduce_row(const double2* __restrict__ part, int k, int G, int B, int b,
                                              int g0, int g1) {
  double re = 0.0, im = 0.0;
  for (int g = g0 + (int)threadIdx.x; g < g1; g += 64) {
    const double2 v = part[((int64_t)k * G + g) * B + b];
    re += v.x;
    im += v.y;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    re += __shfl_xor(re, off);
    im += __shfl_xor(im, off);
  }
  return make_double2(re, im);
}

// One wavefront per (moment k, segment*B + b): sum the segment's workgroup
// partials in a fixed order.  sym: rows hold the raw dots of
// k_moment_step_sym, and moment k >= 2 is 2 raw_k - mu_{k mod 2}.
__global__ __launch_bounds__(64) void k_reduce(const double2* __restrict__ part, int M, int G, int B,
                                               const int32_t* __restrict__ seg_blk0, int sym,
                                               double2* __restrict__ out, double* __restrict__ out_real) {
  const int k = blockIdx.x;
  const int sb = blockIdx.y;
  const int seg = sb / B, b = sb - seg * B;
  const int g0 = seg_blk0[seg], g1 = seg_blk0[seg + 1];
  const double2 v = reduce_row(part, k, G, B, b, g0, g1);
  double re = v.x, im = v.y;
  if (sym && k >= 2) {
    const double2 u = reduce_row(part, k & 1, G, B, b, g0, g1);
    re = 2.0 * re - u.x;
    im = 2.0 * im - u.y;
  }
  if (threadIdx.x == 0) {
    const int64_t o = (int64_t)sb * M + k;
    if (out) out[o] = make_double2(re, im);
    if (out_real) out_real[o] = re;
  }
}

// Transport regimes of Section 2.2 (e = hbar = 1), one energy per thread:
// sigma_sc = max over the rows of the running conductivity (NaN rows skipped),
// v = sqrt(C_vv(E, 0)), tau = sigma_sc / (rho v^2), mfp = v tau,
// L(t) = 2 sqrt(DeltaX^2(t)), xi = L(t_last) / (2 pi); C_vv and DeltaX^2 are the
// reconstructed rows (rho C_vv, rho DeltaX^2) divided by rho.  NaN where rho <= 0,
// C_vv(E, 0) < 0 (v), rho v^2 <= 0 (tau, mfp) or DeltaX^2 < 0 (L, xi).
__global__ __launch_bounds__(256) void k_transport(TransportIO io) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= io.n_E) return;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  const double r = io.rho[e];
  const bool ok = r > 0.0;
  double sc = nan;
  if (io.sigma) {
    for (int k = 0; k < io.n_t; ++k) {
      const double x = io.sigma[(int64_t)k * io.n_E + e];
      if (x == x && (sc != sc || x > sc)) sc = x;
    }
    if (io.sigma_sc) io.sigma_sc[e] = sc;
  }
  if (io.vac0) {
    const double c0 = io.vac0[e];
    const double cvv = ok ? c0 / r : nan;
    const double v = cvv >= 0.0 ? sqrt(cvv) : nan;
    if (io.v) io.v[e] = v;
    if (io.sigma) {
      const double tau = (ok && c0 > 0.0) ? sc / c0 : nan;
      if (io.tau) io.tau[e] = tau;
      if (io.mfp) io.mfp[e] = v * tau;
    }
  }
  if (io.msd) {
    double L = nan;
    for (int k = 0; k < io.n_t; ++k) {
      const double dx2 = ok ? io.msd[(int64_t)k * io.n_E + e] / r : nan;
      L = dx2 >= 0.0 ? 2.0 * sqrt(dx2) : nan;
      if (io.L) io.L[(int64_t)k * io.n_E + e] = L;
    }
    if (io.xi) io.xi[e] = io.n_t > 0 ? L / (2.0 * M_PI) : nan;
  }
}

// Running conductivity (Section 2.2) over the time rows, one energy per thread:
// mode 0 (VAC): trapezoid integral of rows at t_k = sum_{j<k} dt_j, sigma_0 = 0;
// mode 1 (MSD): (y_k - y_{k-1}) / (2 dt_k), y_{-1} = 0 (NaN for dt_k = 0).
__global__ __launch_bounds__(256) void k_sigma(int mode, int n_t, const double* __restrict__ dt, int n_E,
                                               const double* __restrict__ y, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_E) return;
  if (mode == 0) {
    double acc = 0.0, prev = y[e];
    out[e] = 0.0;
    for (int k = 1; k < n_t; ++k) {
      const double cur = y[(int64_t)k * n_E + e];
      acc += 0.5 * dt[k - 1] * (prev + cur);
      out[(int64_t)k * n_E + e] = acc;
      prev = cur;
    }
  } else {
    double prev = 0.0;
    for (int k = 0; k < n_t; ++k) {
      const double cur = y[(int64_t)k * n_E + e];
      out[(int64_t)k * n_E + e] = dt[k] != 0.0 ? (cur - prev) / (2.0 * dt[k]) : __builtin_nan("");
      prev = cur;
    }
  }
}

// KPM sum of Section 3.3 for one (row r, energy e) per thread.  T_n(E~) by the
// Chebyshev recurrence, Jackson damping g_n computed in place.
__global__ __launch_bounds__(256) void k_kpm(int R, int M, const double* __restrict__ C, int n_E,
                                             const double* __restrict__ E, double inv_dE,
                                             double pref_base, int jackson, double cot_pa,
                                             double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (e >= n_E || r >= R) return;
  const double x = E[e] * inv_dE;
  if (!(fabs(x) < 1.0)) {
    out[(int64_t)r * n_E + e] = __builtin_nan("");
    return;
  }
  const double a = 1.0 / (M + 1);
  const double* c = C + (int64_t)r * M;
  double t0 = 1.0, t1 = x, s = c[0];
  for (int n = 1; n < M; ++n) {
    double g = 1.0;
    if (jackson) {
      double sn, cs;
      sincospi(n * a, &sn, &cs);
      g = (1.0 - n * a) * cs + a * sn * cot_pa;
    }
    s += 2.0 * g * t1 * c[n];
    const double t2 = 2.0 * x * t1 - t0;
    t0 = t1;
    t1 = t2;
  }
  out[(int64_t)r * n_E + e] = pref_base / sqrt(1.0 - x * x) * s;
}

// Transpose of k_kpm: out[r][n] = sum_e g[r][e] pref(E_e) w_n T_n(E~_e), one (row r,
// moment n) per thread; energies outside the band contribute nothing.
__global__ __launch_bounds__(256) void k_kpm_adjoint(int R, int M, const double* __restrict__ g, int n_E,
                                                     const double* __restrict__ E, double inv_dE,
                                                     double pref_base, int jackson, double cot_pa,
                                                     double* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (n >= M || r >= R) return;
  const double a = 1.0 / (M + 1);
  double wn = n == 0 ? 1.0 : 2.0;
  if (jackson && n > 0) {
    double sn, cs;
    sincospi(n * a, &sn, &cs);
    wn *= (1.0 - n * a) * cs + a * sn * cot_pa;
  }
  double s = 0.0;
  for (int e = 0; e < n_E; ++e) {
    const double x = E[e] * inv_dE;
    if (!(fabs(x) < 1.0)) continue;
    s += g[(int64_t)r * n_E + e] * pref_base / sqrt(1.0 - x * x) * cos(n * acos(x));
  }
  out[(int64_t)r * M + n] = wn * s;
}

// Bandwidth probe: one 16-byte element per thread over a grid that covers the
// whole buffer (every element's load is in flight at once, as far as the chip
// holds them; no loop-carried address arithmetic).
__global__ __launch_bounds__(256) void k_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                              size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace


// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

int kernel_occupancy(int family, const DevMat& A, int hop_mode, int B, int nt) {
  int nb = 0;
  auto q = [&](auto fn) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kBlock, 0) != hipSuccess) nb = 0;
  };
  (void)dispatch_sparse(A, hop_mode, B, nt, [&](auto Bc, auto Hc, auto Kc, auto NTc) {
    constexpr int b = decltype(Bc)::value, hm = decltype(Hc)::value, k = decltype(Kc)::value;
    constexpr bool n = decltype(NTc)::value;
    switch (family) {
      case FAM_MOMENT: q(k_moment_step<b, hm, k, n>); break;
      case FAM_SYM: q(k_moment_step_sym<b, hm, k, n>); break;
      case FAM_PAIR: q(k_moment_step_pair<b, hm, k, n>); break;
      case FAM_EVOLVE: q(k_evolve_term<b, hm, k, n>); break;
      case FAM_EVOLVE_PAIR: q(k_evolve_pair_term<b, hm, k, n>); break;
      default: q(k_msd_term<b, hm, k, n>); break;
    }
  });
  (void)hipGetLastError();
  return nb;
}

hipError_t launch_moment_step(const DevMat& A, int hop_mode, int B, const StepIO& io,
                              const double2* phiL, double2* part_n, double2* part_0, hipStream_t s) {
  return dispatch_sparse(A, hop_mode, B, A.nt, [&](auto Bc, auto Hc, auto Kc, auto NTc) {
    k_moment_step<decltype(Bc)::value, decltype(Hc)::value, decltype(Kc)::value, decltype(NTc)::value>
        <<<dim3(A.G), kBlock, 0, s>>>(A, io, phiL, part_n, part_0);
  });
}

hipError_t launch_evolve_term(const DevMat& A, int hop_mode, int B, const StepIO& io, double2* acc,
                              const double* Jtab, int ldJ, int m, double2 phase_m, double2 phase_0,
                              hipStream_t s) {
  return dispatch_sparse(A, hop_mode, B, A.nt, [&](auto Bc, auto Hc, auto Kc, auto NTc) {
    k_evolve_term<decltype(Bc)::value, decltype(Hc)::value, decltype(Kc)::value, decltype(NTc)::value>
        <<<dim3(A.G), kBlock, 0, s>>>(A, io, acc, Jtab, ldJ, m, phase_m, phase_0);
  });
}

namespace {

// The fused MSD term of k_msd_term on a periodic box whose position differences are
// +-box_dx on the x neighbours and 0 on the others, as the box stencil of
// k_moment_step_sym_box with both chains staged: [X,H~] a at a row is
// -box_dx hu (a_{x+1} - a_{x-1}).  Work items, tiles, addressing and the one-plane
// lookahead as there; no partial sums.
template <int B, int TX, int TY, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_msd_term_box(DevMat A, ChainIO io, double2* acc_a, double2* acc_b,
                                                         const double* __restrict__ Jtab, int ldJ, int m,
                                                         double2 ph_m, double2 ph_0, int zc) {
  using T = BoxTile<B, TX, TY>;
  constexpr int OPT = T::OPT, HPT = T::HPT, PX = T::PX;
  __shared__ double2 lda[2][T::PE], ldb[2][T::PE];
  const int lb = logical_block(A.G);
  const int Lx = A.box[0], Ly = A.box[1], Lz = A.box[2];
  const int txn = (Lx + TX - 1) / TX, tyn = (Ly + TY - 1) / TY, zn = (Lz + zc - 1) / zc;
  const int64_t cols = (int64_t)txn * tyn, items = cols * zn;
  const double hu = A.seg_hop[0];
  const double hdx = hu * A.box_dx;
  const double2 cm = cscale(Jtab[m], ph_m);
  const double2 c0 = cscale(Jtab[0], ph_0);
  const int b = threadIdx.x & (B - 1);
  const char* xas = reinterpret_cast<const char*>(io.xa);
  const char* xbs = reinterpret_cast<const char*>(io.xb);
  // read only after the first step: the previous chain elements and the running sums
  // (acc is read and then overwritten element by element, so it is not restrict)
  const char* was = reinterpret_cast<const char*>(io.wa);
  const char* wbs = reinterpret_cast<const char*>(io.wb);
  const char* sas = reinterpret_cast<const char*>(acc_a);
  const char* sbs = reinterpret_cast<const char*>(acc_b);
  char* oas = reinterpret_cast<char*>(io.oa);
  char* obs = reinterpret_cast<char*>(io.ob);
  char* aas = reinterpret_cast<char*>(acc_a);
  char* abs_ = reinterpret_cast<char*>(acc_b);
  const char* ds = reinterpret_cast<const char*>(A.diag);
  const int64_t vplane = (int64_t)Lx * Ly * B * (int64_t)sizeof(double2);
  const int64_t dplane = (int64_t)Lx * Ly * (int64_t)sizeof(double);
  auto zw = [Lz](int z) { return z < 0 ? z + Lz : (z >= Lz ? z - Lz : z); };   // z in [-1, Lz + 1]
  T t(b);
  for (int64_t it = lb; it < items; it += A.G) {
    const int tz = (int)(it / cols);
    const int64_t txy = it % cols;
    const int z0 = tz * zc, z1 = min(z0 + zc, Lz);
    t.place((int)(txy % txn) * TX, (int)(txy / txn) * TY, Lx, Ly, b);
    // chains a and b of planes z - 1, z, z + 1 and the ones loaded for z + 2 rotate through
    // a0..a3 and b0..b3; the previous chain elements, the running sums, the diagonal and the
    // halos of planes z and z + 1 through pairs; unrolled four planes deep as in
    // k_moment_step_sym_box, so that the rotation is a renaming
    double2 a0[OPT], a1[OPT], a2[OPT], a3[OPT], b0[OPT], b1[OPT], b2[OPT], b3[OPT];
    double2 wa0[OPT], wa1[OPT], wb0[OPT], wb1[OPT], sa0[OPT], sa1[OPT], sb0[OPT], sb1[OPT];
    double d0[OPT], d1[OPT];
    double2 ha0[HPT], ha1[HPT], hb0[HPT], hb1[HPT];
    // the once-read operands of plane z (only the diagonal on the first step)
    auto ld_prev = [&](int z, double2(&wa)[OPT], double2(&wb)[OPT], double2(&sa)[OPT], double2(&sb)[OPT],
                       double(&d)[OPT]) {
      const int64_t v = z * vplane;
#pragma unroll
      for (int i = 0; i < OPT; ++i) {
        if (!FIRST) {
          wa[i] = box_ld<kBoxNtLoad>(was + v, t.oo[i]);
          wb[i] = box_ld<kBoxNtLoad>(wbs + v, t.oo[i]);
          sa[i] = box_ld<kBoxNtLoad>(sas + v, t.oo[i]);
          sb[i] = box_ld<kBoxNtLoad>(sbs + v, t.oo[i]);
        }
        d[i] = box_ldd(ds + z * dplane, t.od[i]);
      }
    };
    {
      const int64_t vm = zw(z0 - 1) * vplane, v0 = z0 * vplane, vp = zw(z0 + 1) * vplane;
#pragma unroll
      for (int i = 0; i < OPT; ++i) {
        wa0[i] = wb0[i] = sa0[i] = sb0[i] = make_double2(0.0, 0.0);
        wa1[i] = wb1[i] = sa1[i] = sb1[i] = make_double2(0.0, 0.0);
        a0[i] = box_ld(xas + vm, t.oo[i]);
        a1[i] = box_ld(xas + v0, t.oo[i]);
        a2[i] = box_ld(xas + vp, t.oo[i]);
        b0[i] = box_ld(xbs + vm, t.oo[i]);
        b1[i] = box_ld(xbs + v0, t.oo[i]);
        b2[i] = box_ld(xbs + vp, t.oo[i]);
      }
      ld_prev(z0, wa0, wb0, sa0, sb0, d0);
#pragma unroll
      for (int j = 0; j < HPT; ++j) {
        ha0[j] = box_ld(xas + v0, t.ho[j]);
        hb0[j] = box_ld(xbs + v0, t.ho[j]);
      }
    }
    // plane z in LDS buffer BF: the loads for plane z + 1 (unconditional, as in
    // k_moment_step_sym_box), then the stencil on both chains
    auto plane = [&](int z, auto BF, double2(&am)[OPT], double2(&ac)[OPT], double2(&ap)[OPT], double2(&aq)[OPT],
                     double2(&bm)[OPT], double2(&bc)[OPT], double2(&bp)[OPT], double2(&bq)[OPT],
                     double2(&wac)[OPT], double2(&wan)[OPT], double2(&wbc)[OPT], double2(&wbn)[OPT],
                     double2(&sac)[OPT], double2(&san)[OPT], double2(&sbc)[OPT], double2(&sbn)[OPT],
                     double(&dc)[OPT], double(&dn)[OPT], double2(&hac)[HPT], double2(&han)[HPT],
                     double2(&hbc)[HPT], double2(&hbn)[HPT]) {
      constexpr int bf = decltype(BF)::value;
      {
        const int z1n = zw(z + 1);
        const int64_t vq = zw(z + 2) * vplane, vn = z1n * vplane;
#pragma unroll
        for (int i = 0; i < OPT; ++i) {
          aq[i] = box_ld(xas + vq, t.oo[i]);
          bq[i] = box_ld(xbs + vq, t.oo[i]);
        }
        ld_prev(z1n, wan, wbn, san, sbn, dn);
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
          han[j] = box_ld(xas + vn, t.ho[j]);
          hbn[j] = box_ld(xbs + vn, t.ho[j]);
        }
      }
#pragma unroll
      for (int i = 0; i < OPT; ++i) {
        lda[bf][t.oslot[i]] = ac[i];
        ldb[bf][t.oslot[i]] = bc[i];
      }
#pragma unroll
      for (int j = 0; j < HPT; ++j)
        if (t.hval[j]) {
          lda[bf][t.hslot[j]] = hac[j];
          ldb[bf][t.hslot[j]] = hbc[j];
        }
      __syncthreads();
      const int64_t vz = z * vplane;
#pragma unroll
      for (int i = 0; i < OPT; ++i) {
        if (t.oval[i]) {
          const int c = t.oslot[i];
          const double2 axp = lda[bf][c + B], axm = lda[bf][c - B];
          double2 na = cadd(axp, axm);
          na = cadd(na, lda[bf][c + PX * B]);
          na = cadd(na, lda[bf][c - PX * B]);
          na = cadd(na, ap[i]);
          na = cadd(na, am[i]);
          double2 nb = cadd(ldb[bf][c + B], ldb[bf][c - B]);
          nb = cadd(nb, ldb[bf][c + PX * B]);
          nb = cadd(nb, ldb[bf][c - PX * B]);
          nb = cadd(nb, bp[i]);
          nb = cadd(nb, bm[i]);
          const double dg = dc[i];
          const double2 ha = make_double2(fma(dg, ac[i].x, hu * na.x), fma(dg, ac[i].y, hu * na.y));
          const double2 hb = make_double2(fma(dg, bc[i].x, hu * nb.x), fma(dg, bc[i].y, hu * nb.y));
          // [X,H~] a + H~ b, [X,H~]_rj = -dx_rj H~_rj
          const double2 g = make_double2(hb.x - hdx * (axp.x - axm.x), hb.y - hdx * (axp.y - axm.y));
          if (FIRST) {
            box_st(oas + vz, t.oo[i], ha);
            box_st(obs + vz, t.oo[i], g);
            box_st(aas + vz, t.oo[i], cadd(cmul(c0, ac[i]), cmul(cm, ha)));
            box_st(abs_ + vz, t.oo[i], cadd(cmul(c0, bc[i]), cmul(cm, g)));
          } else {
            const double2 ya = twice_minus(ha, wac[i]);
            const double2 yb = twice_minus(g, wbc[i]);
            box_st(oas + vz, t.oo[i], ya);
            box_st(obs + vz, t.oo[i], yb);
            box_st(aas + vz, t.oo[i], cadd(sac[i], cmul(cm, ya)));
            box_st(abs_ + vz, t.oo[i], cadd(sbc[i], cmul(cm, yb)));
          }
        }
      }
    };
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    for (int z = z0; z < z1; z += 4) {
      plane(z, S0{}, a0, a1, a2, a3, b0, b1, b2, b3, wa0, wa1, wb0, wb1, sa0, sa1, sb0, sb1, d0, d1, ha0, ha1,
            hb0, hb1);
      if (z + 1 >= z1) break;
      plane(z + 1, S1{}, a1, a2, a3, a0, b1, b2, b3, b0, wa1, wa0, wb1, wb0, sa1, sa0, sb1, sb0, d1, d0, ha1,
            ha0, hb1, hb0);
      if (z + 2 >= z1) break;
      plane(z + 2, S0{}, a2, a3, a0, a1, b2, b3, b0, b1, wa0, wa1, wb0, wb1, sa0, sa1, sb0, sb1, d0, d1, ha0,
            ha1, hb0, hb1);
      if (z + 3 >= z1) break;
      plane(z + 3, S1{}, a3, a0, a1, a2, b3, b0, b1, b2, wa1, wa0, wb1, wb0, sa1, sa0, sb1, sb0, d1, d0, ha1,
            ha0, hb1, hb0);
    }
    __syncthreads();   // the next item stages into buffer 0 again
  }
}

}  // namespace

// Planes per work item of the box kernels on tiles of tx x ty (stencil_run over the G
// workgroups).
static int box_run(const DevMat& A, int tx, int ty) {
  const int64_t cols = (int64_t)((A.box[0] + tx - 1) / tx) * ((A.box[1] + ty - 1) / ty);
  return stencil_run(cols, A.box[2], A.G);
}

hipError_t launch_msd_term(const DevMat& A, int hop_mode, int B, const ChainIO& io, double2* acc_a,
                           double2* acc_b, const double* Jtab, int ldJ, int m, double2 phase_m,
                           double2 phase_0, hipStream_t s) {
  if (A.use_box_msd && A.box[0] > 0 && hop_mode == HOP_UNIFORM && B >= 2) {
    // tiles: 16 x 8 (B = 2), 8 x 8 (4), 8 x 4 (8), 4 x 4 (16): two staged chains fit the LDS
    const int zc = box_run(A, B == 2 ? 16 : (B == 16 ? 4 : 8), B >= 8 ? 4 : 8);
    auto go = [&](auto Fc) {
      constexpr bool F = decltype(Fc)::value;
      const dim3 g(A.G);
      switch (B) {
        case 2: k_msd_term_box<2, 16, 8, F><<<g, kBlock, 0, s>>>(A, io, acc_a, acc_b, Jtab, ldJ, m, phase_m, phase_0, zc); break;
        case 4: k_msd_term_box<4, 8, 8, F><<<g, kBlock, 0, s>>>(A, io, acc_a, acc_b, Jtab, ldJ, m, phase_m, phase_0, zc); break;
        case 8: k_msd_term_box<8, 8, 4, F><<<g, kBlock, 0, s>>>(A, io, acc_a, acc_b, Jtab, ldJ, m, phase_m, phase_0, zc); break;
        default: k_msd_term_box<16, 4, 4, F><<<g, kBlock, 0, s>>>(A, io, acc_a, acc_b, Jtab, ldJ, m, phase_m, phase_0, zc); break;
      }
    };
    if (io.first) go(std::true_type{}); else go(std::false_type{});
    return hipGetLastError();
  }
  return dispatch_sparse(A, hop_mode, B, A.nt, [&](auto Bc, auto Hc, auto Kc, auto NTc) {
    k_msd_term<decltype(Bc)::value, decltype(Hc)::value, decltype(Kc)::value, decltype(NTc)::value>
        <<<dim3(A.G), kBlock, 0, s>>>(A, io, acc_a, acc_b, Jtab, ldJ, m, phase_m, phase_0);
  });
}

hipError_t launch_evolve_pair_term(const DevMat& A, int hop_mode, int B, const ChainIO& io, double2* acc_a,
                                   double2* acc_b, const double* Jtab, int ldJ, int m, double2 phase_m,
                                   double2 phase_0, hipStream_t s) {
  return dispatch_sparse(A, hop_mode, B, A.nt, [&](auto Bc, auto Hc, auto Kc, auto NTc) {
    k_evolve_pair_term<decltype(Bc)::value, decltype(Hc)::value, decltype(Kc)::value, decltype(NTc)::value>
        <<<dim3(A.G), kBlock, 0, s>>>(A, io, acc_a, acc_b, Jtab, ldJ, m, phase_m, phase_0);
  });
}

hipError_t launch_commutator(const DevMat& A, int hop_mode, int B, int which, const double2* x,
                             double2* out, hipStream_t s) {
  return dispatch_bh(B, hop_mode, [&](auto Bc, auto Hc) {
    k_commutator<decltype(Bc)::value, decltype(Hc)::value><<<dim3(A.G), kBlock, 0, s>>>(A, which, x, out);
  });
}

hipError_t launch_scale(const DevMat& A, int B, const double2* in, double2* out, const double* Jtab,
                        int ldJ, hipStream_t s) {
  return dispatch_bh(B, HOP_UNIFORM, [&](auto Bc, auto) {
    k_scale<decltype(Bc)::value><<<dim3(A.G), kBlock, 0, s>>>(A, in, out, Jtab, ldJ);
  });
}

hipError_t launch_fill_phase(const DevMat& A, int B, double2* out, hipStream_t s) {
  return dispatch_bh(B, HOP_UNIFORM, [&](auto Bc, auto) {
    k_fill_phase<decltype(Bc)::value><<<dim3(A.G), kBlock, 0, s>>>(A, out);
  });
}

hipError_t launch_bessel_table(const double* seg_dE, int n_seg, double abs_dt, int Np, int ldJ,
                               double* J, hipStream_t s) {
  const int threads = 64;
  const int blocks = (n_seg + threads - 1) / threads;
  k_bessel_table<<<blocks, threads, 0, s>>>(seg_dE, n_seg, abs_dt, Np, ldJ, J);
  return hipGetLastError();
}

hipError_t launch_reduce_moments(const double2* part, int M, int G, int B, int n_seg,
                                 const int32_t* seg_blk0_dev, int sym, double2* out, double* out_real,
                                 hipStream_t s) {
  if (M <= 0) return hipSuccess;
  k_reduce<<<dim3(M, n_seg * B), 64, 0, s>>>(part, M, G, B, seg_blk0_dev, sym, out, out_real);
  return hipGetLastError();
}

hipError_t launch_moment_step_pair(const DevMat& A, int hop_mode, int B, const ChainIO& io,
                                   double2* part_a, double2* part_b, double2* part_c, hipStream_t s) {
  return dispatch_sparse(A, hop_mode, B, A.nt, [&](auto Bc, auto Hc, auto Kc, auto NTc) {
    k_moment_step_pair<decltype(Bc)::value, decltype(Hc)::value, decltype(Kc)::value,
                       decltype(NTc)::value><<<dim3(A.G), kBlock, 0, s>>>(A, io, part_a, part_b, part_c);
  });
}

hipError_t launch_moment_step_sym(const DevMat& A, int hop_mode, int B, const StepIO& io,
                                  double2* part_a, double2* part_b, double2* part_c, hipStream_t s) {
  if (A.use_sheet && A.sheet && A.sheet_zc && A.sheet_blk0 && hop_mode == HOP_UNIFORM && B >= 2) {
    auto go = [&](auto Fc) {
      constexpr bool F = decltype(Fc)::value;
      const dim3 g(A.G);
      switch (B) {
        case 2: k_moment_step_sym_sheet<2, kSheetCells, F><<<g, kBlock, 0, s>>>(A, io, part_a, part_b, part_c); break;
        case 4: k_moment_step_sym_sheet<4, kSheetCells, F><<<g, kBlock, 0, s>>>(A, io, part_a, part_b, part_c); break;
        case 8: k_moment_step_sym_sheet<8, kSheetCells, F><<<g, kBlock, 0, s>>>(A, io, part_a, part_b, part_c); break;
        default: k_moment_step_sym_sheet<16, kSheetCells, F><<<g, kBlock, 0, s>>>(A, io, part_a, part_b, part_c); break;
      }
    };
    if (io.first) go(std::true_type{}); else go(std::false_type{});
    return hipGetLastError();
  }
  if (A.use_box && A.box[0] > 0 && hop_mode == HOP_UNIFORM && B >= 2) {
    const int zc = box_run(A, B == 2 ? 16 : 8, 8);   // the tiles of the instances below
    auto go = [&](auto Fc) {
      constexpr bool F = decltype(Fc)::value;
      const dim3 g(A.G);
      switch (B) {
        case 2: k_moment_step_sym_box<2, 16, 8, F><<<g, kBlock, 0, s>>>(A, io, zc, part_a, part_b, part_c); break;
        case 4: k_moment_step_sym_box<4, 8, 8, F><<<g, kBlock, 0, s>>>(A, io, zc, part_a, part_b, part_c); break;
        case 8: k_moment_step_sym_box<8, 8, 8, F><<<g, kBlock, 0, s>>>(A, io, zc, part_a, part_b, part_c); break;
        default: k_moment_step_sym_box<16, 8, 8, F><<<g, kBlock, 0, s>>>(A, io, zc, part_a, part_b, part_c); break;
      }
    };
    if (io.first) go(std::true_type{}); else go(std::false_type{});
    return hipGetLastError();
  }
  return dispatch_sparse(A, hop_mode, B, A.nt, [&](auto Bc, auto Hc, auto Kc, auto NTc) {
    k_moment_step_sym<decltype(Bc)::value, decltype(Hc)::value, decltype(Kc)::value,
                      decltype(NTc)::value><<<dim3(A.G), kBlock, 0, s>>>(A, io, part_a, part_b, part_c);
  });
}

hipError_t launch_kpm(int R, int M, const double* C, int n_E, const double* E, double inv_dE,
                      double pref_base, int jackson, double* out, hipStream_t s) {
  if (R <= 0 || n_E <= 0) return hipSuccess;
  const double a = 1.0 / (M + 1);
  const double cot_pa = cos(M_PI * a) / sin(M_PI * a);
  k_kpm<<<dim3((n_E + 255) / 256, R), 256, 0, s>>>(R, M, C, n_E, E, inv_dE, pref_base, jackson, cot_pa,
                                                   out);
  return hipGetLastError();
}

hipError_t launch_kpm_adjoint(int R, int M, const double* g, int n_E, const double* E, double inv_dE,
                              double pref_base, int jackson, double* out, hipStream_t s) {
  if (R <= 0 || M <= 0) return hipSuccess;
  const double a = 1.0 / (M + 1);
  const double cot_pa = cos(M_PI * a) / sin(M_PI * a);
  k_kpm_adjoint<<<dim3((M + 255) / 256, R), 256, 0, s>>>(R, M, g, n_E, E, inv_dE, pref_base, jackson,
                                                         cot_pa, out);
  return hipGetLastError();
}

hipError_t launch_transport(const TransportIO& io, hipStream_t s) {
  if (io.n_E <= 0) return hipSuccess;
  k_transport<<<dim3((io.n_E + 255) / 256), 256, 0, s>>>(io);
  return hipGetLastError();
}

hipError_t launch_sigma(int mode, int n_t, const double* dt, int n_E, const double* y, double* out,
                        hipStream_t s) {
  if (n_t <= 0 || n_E <= 0) return hipSuccess;
  k_sigma<<<dim3((n_E + 255) / 256), 256, 0, s>>>(mode, n_t, dt, n_E, y, out);
  return hipGetLastError();
}

hipError_t launch_copy(const double2* src, double2* dst, size_t n16, hipStream_t s) {
  if (n16 == 0) return hipSuccess;
  const size_t blocks = (n16 + 255) / 256;
  if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
  k_copy<<<dim3((unsigned)blocks), 256, 0, s>>>(src, dst, n16);
  return hipGetLastError();
}

}  // namespace gpuqt
