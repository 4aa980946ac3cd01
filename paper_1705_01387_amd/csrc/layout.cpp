// Host-side validation of a tight-binding descriptor and construction of the
// sliced-ELL layout (pure C++, no device calls).
//
// The model is the one the paper's input files describe (Section 4.2):
// neighbour list, hoppings (default -1), on-site potentials (default 0),
// positions along the transport direction with the period used for bonds
// across the boundary.  The spectrum of H / DeltaE must lie in [-1, 1]
// (Section 3.2); DeltaE is checked against the Gershgorin bound
// max_i (|U_i| + sum_j |H_ij|), which contains every eigenvalue.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <unordered_map>

#include "internal.h"

namespace gpuqt {

namespace {

struct Bond {
  int64_t i, j;
  double re, im;
};

bool check_hermitian(const std::vector<Bond>& bonds, const std::vector<double>& diag_im,
                     std::string* msg) {
  // Sum duplicates, then require H_ji = conj(H_ij) for every stored pair.
  std::vector<Bond> b = bonds;
  std::sort(b.begin(), b.end(), [](const Bond& p, const Bond& q) {
    return p.i != q.i ? p.i < q.i : p.j < q.j;
  });
  std::vector<Bond> u;
  u.reserve(b.size());
  double scale = 0.0;
  for (const Bond& x : b) {
    if (!u.empty() && u.back().i == x.i && u.back().j == x.j) {
      u.back().re += x.re;
      u.back().im += x.im;
    } else {
      u.push_back(x);
    }
  }
  for (const Bond& x : u) scale = std::max(scale, std::hypot(x.re, x.im));
  const double tol = 1e-12 * std::max(scale, 1e-300);
  for (const Bond& x : u) {
    if (x.i == x.j) {
      if (std::fabs(x.im) > tol) {
        *msg = "self-bond of orbital " + std::to_string(x.i) + " is not real";
        return false;
      }
      continue;
    }
    auto it = std::lower_bound(u.begin(), u.end(), x, [](const Bond& p, const Bond& q) {
      return p.i != q.j ? p.i < q.j : p.j < q.i;
    });
    double re = 0.0, im = 0.0;
    if (it != u.end() && it->i == x.j && it->j == x.i) {
      re = it->re;
      im = it->im;
    }
    if (std::fabs(re - x.re) > tol || std::fabs(im + x.im) > tol) {
      *msg = "H is not Hermitian: H[" + std::to_string(x.i) + "," + std::to_string(x.j) +
             "] has no conjugate partner H[" + std::to_string(x.j) + "," +
             std::to_string(x.i) + "]";
      return false;
    }
  }
  (void)diag_im;
  return true;
}

}  // namespace

gpuqt_status build_host_layout(const gpuqt_h_desc* d, HostLayout* L, std::string* msg) {
  if (!d) {
    *msg = "desc is NULL";
    return GPUQT_ERR_ARG;
  }
  if (d->n < 1) {
    *msg = "n must be >= 1";
    return GPUQT_ERR_ARG;
  }
  if (d->n > (int64_t)INT32_MAX) {
    *msg = "n must fit a 32-bit neighbour index";
    return GPUQT_ERR_UNSUPPORTED;
  }
  if (d->max_nn < 0 || d->max_nn > 4096) {
    *msg = "max_nn must be in [0, 4096]";
    return GPUQT_ERR_ARG;
  }
  if (!d->nn || !d->x || (d->max_nn > 0 && !d->nbr)) {
    *msg = "nn, x (and nbr when max_nn > 0) are required";
    return GPUQT_ERR_ARG;
  }
  const int32_t n_class = d->n_class < 1 ? 1 : d->n_class;
  if (d->hop_class && d->n_class < 1) {
    *msg = "n_class must be >= 1 when hop_class is given";
    return GPUQT_ERR_ARG;
  }
  int S = d->slice_height == 0 ? 64 : d->slice_height;
  if (S < 32 || S > 1024 || (S & (S - 1))) {
    *msg = "slice_height must be 0 or a power of two in [32, 1024]";
    return GPUQT_ERR_ARG;
  }
  if (d->band_rows < 0 || d->band_rows % 64 != 0) {
    *msg = "band_rows must be 0 or a positive multiple of 64";
    return GPUQT_ERR_ARG;
  }
  const int64_t n = d->n;
  const int k = d->max_nn;

  // segments
  const int32_t n_seg = d->n_segments > 1 ? d->n_segments : 1;
  std::vector<int64_t> seg_off(n_seg + 1);
  if (n_seg > 1) {
    if (!d->seg_offsets) {
      *msg = "seg_offsets is required when n_segments > 1";
      return GPUQT_ERR_ARG;
    }
    for (int s = 0; s <= n_seg; ++s) seg_off[s] = d->seg_offsets[s];
    if (seg_off[0] != 0 || seg_off[n_seg] != n) {
      *msg = "seg_offsets must start at 0 and end at n";
      return GPUQT_ERR_ARG;
    }
    for (int s = 0; s < n_seg; ++s)
      if (seg_off[s + 1] <= seg_off[s]) {
        *msg = "seg_offsets must be strictly increasing";
        return GPUQT_ERR_ARG;
      }
  } else {
    seg_off[0] = 0;
    seg_off[1] = n;
  }

  // neighbour list checks, position differences, Gershgorin per segment
  std::vector<double> gersh(n_seg, 0.0);
  std::vector<int32_t> seg_of_row(n);
  for (int s = 0; s < n_seg; ++s)
    for (int64_t i = seg_off[s]; i < seg_off[s + 1]; ++i) seg_of_row[i] = s;
  const bool cplx = d->hop && d->hop_is_complex;
  std::vector<double> rowsum(n, 0.0);
  std::vector<Bond> bonds;
  if (d->check_hermitian) bonds.reserve((size_t)n * (size_t)k);
  bool any_imag = false;
  int64_t nnz = 0;
  int32_t max_deg = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t c = d->nn[i];
    if (c < 0 || c > k) {
      *msg = "neighbour count of orbital " + std::to_string(i) + " is " + std::to_string(c) +
             ", outside [0, max_nn]";
      return GPUQT_ERR_LAYOUT;
    }
    max_deg = std::max(max_deg, c);
    nnz += c;
    const int s = seg_of_row[i];
    for (int j = 0; j < c; ++j) {
      const int64_t e = i * k + j;
      const int64_t col = d->nbr[e];
      if (col < 0 || col >= n) {
        *msg = "neighbour " + std::to_string(j) + " of orbital " + std::to_string(i) +
               " is " + std::to_string(col) + ", outside [0, n)";
        return GPUQT_ERR_LAYOUT;
      }
      if (col < seg_off[s] || col >= seg_off[s + 1]) {
        *msg = "bond " + std::to_string(i) + "-" + std::to_string(col) + " joins two segments";
        return GPUQT_ERR_LAYOUT;
      }
      double re = -1.0, im = 0.0;
      if (d->hop) {
        if (cplx) {
          re = d->hop[2 * e];
          im = d->hop[2 * e + 1];
        } else {
          re = d->hop[e];
        }
      }
      if (!std::isfinite(re) || !std::isfinite(im)) {
        *msg = "hopping " + std::to_string(j) + " of orbital " + std::to_string(i) +
               " is not finite";
        return GPUQT_ERR_ARG;
      }
      if (im != 0.0) any_imag = true;
      if (d->hop_class) {
        const int32_t cl = d->hop_class[e];
        if (cl < 0 || cl >= n_class) {
          *msg = "hop_class of bond " + std::to_string(i) + "-" + std::to_string(col) +
                 " is outside [0, n_class)";
          return GPUQT_ERR_ARG;
        }
      }
      rowsum[i] += std::hypot(re, im);
      if (d->check_hermitian) bonds.push_back({i, col, re, im});
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    const double u = d->onsite ? d->onsite[i] : 0.0;
    if (!std::isfinite(u) || !std::isfinite(d->x[i])) {
      *msg = "on-site energy or position of orbital " + std::to_string(i) + " is not finite";
      return GPUQT_ERR_ARG;
    }
    const int s = seg_of_row[i];
    gersh[s] = std::max(gersh[s], std::fabs(u) + rowsum[i]);
  }
  if (d->check_hermitian && !check_hermitian(bonds, {}, msg)) return GPUQT_ERR_LAYOUT;
  bonds.clear();
  bonds.shrink_to_fit();

  // DeltaE per segment
  std::vector<double> dE(n_seg);
  for (int s = 0; s < n_seg; ++s) {
    double v = d->energy_max;
    if (d->seg_energy_max && d->seg_energy_max[s] > 0) v = d->seg_energy_max[s];
    if (!(v > 0)) v = gersh[s] > 0 ? 1.01 * gersh[s] : 1.0;
    if (!std::isfinite(v)) {
      *msg = "energy_max is not finite";
      return GPUQT_ERR_ARG;
    }
    if (v < gersh[s] * (1.0 - 1e-12)) {
      *msg = "energy_max " + std::to_string(v) + " of segment " + std::to_string(s) +
             " is below the Gershgorin bound " + std::to_string(gersh[s]) +
             ": the spectrum of H/DeltaE may leave [-1, 1]";
      return GPUQT_ERR_SPECTRUM;
    }
    dE[s] = v;
  }

  // hopping storage mode: one value per segment when every hopping of the
  // segment is the same real number (always so for the paper's default -1)
  int mode = cplx && any_imag ? HOP_COMPLEX : HOP_REAL;
  std::vector<double> seg_hop(n_seg, 0.0);
  if (mode == HOP_REAL && n_class == 1) {
    bool uniform = true;
    std::vector<int> seen(n_seg, 0);
    for (int64_t i = 0; i < n && uniform; ++i) {
      const int s = seg_of_row[i];
      for (int j = 0; j < d->nn[i]; ++j) {
        const int64_t e = i * k + j;
        const double h = d->hop ? (cplx ? d->hop[2 * e] : d->hop[e]) : -1.0;
        if (!seen[s]) {
          seen[s] = 1;
          seg_hop[s] = h;
        } else if (h != seg_hop[s]) {
          uniform = false;
          break;
        }
      }
    }
    if (uniform) mode = HOP_UNIFORM;
  }
  for (int s = 0; s < n_seg; ++s) seg_hop[s] /= dE[s];

  // sliced ELL
  int S_log2 = 0;
  while ((1 << S_log2) < S) ++S_log2;
  const int64_t n_slices = (n + S - 1) / S;
  std::vector<int64_t> slice_ptr(n_slices + 1, 0);
  int32_t max_w = 0;
  for (int64_t s = 0; s < n_slices; ++s) {
    int32_t w = 0;
    const int64_t r1 = std::min<int64_t>(n, (s + 1) * S);
    for (int64_t i = s * S; i < r1; ++i) w = std::max(w, d->nn[i]);
    max_w = std::max(max_w, w);
    slice_ptr[s + 1] = slice_ptr[s] + (int64_t)w * S;
  }
  bool unif_w = true;
  for (int64_t i = 0; i < n; ++i)
    if (d->nn[i] != max_deg) {
      unif_w = false;
      break;
    }
  const int64_t entries = slice_ptr[n_slices];
  L->col.assign(entries, -1);
  L->dx.assign(entries, 0.0);
  if (mode == HOP_REAL) L->hop.assign(entries, 0.0);
  if (mode == HOP_COMPLEX) L->hop.assign(2 * entries, 0.0);
  if (d->hop_class && n_class > 1) L->cls.assign(entries, -1);
  L->diag.assign(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    const int seg = seg_of_row[i];
    const double Lx = d->seg_length_x ? d->seg_length_x[seg] : d->length_x;
    const int64_t sl = i >> S_log2;
    const int64_t base = slice_ptr[sl] + (i & (S - 1));
    const double inv = 1.0 / dE[seg];
    L->diag[i] = (d->onsite ? d->onsite[i] : 0.0) * inv;
    for (int j = 0; j < d->nn[i]; ++j) {
      const int64_t e = i * k + j;
      const int64_t slot = base + (int64_t)j * S;
      const int32_t col = d->nbr[e];
      L->col[slot] = col;
      double dxv = d->x[col] - d->x[i];
      if (Lx > 0) {
        const double img = dxv - Lx * std::round(dxv / Lx);
        if (std::fabs(std::fabs(img) - 0.5 * Lx) <= 1e-9 * Lx) {
          *msg = "bond " + std::to_string(i) + "-" + std::to_string(col) +
                 " spans half the period: its direction across the boundary is ambiguous";
          return GPUQT_ERR_LAYOUT;
        }
        dxv = img;
      }
      L->dx[slot] = dxv;
      if (mode == HOP_REAL) L->hop[slot] = (d->hop ? (cplx ? d->hop[2 * e] : d->hop[e]) : -1.0) * inv;
      if (mode == HOP_COMPLEX) {
        L->hop[2 * slot] = d->hop[2 * e] * inv;
        L->hop[2 * slot + 1] = d->hop[2 * e + 1] * inv;
      }
      if (!L->cls.empty()) L->cls[slot] = d->hop_class[e];
    }
  }

  // value table (at most 4 hopping classes, few distinct (column offset, hopping,
  // dx, class) tuples); not for one uniform hopping per segment: there the column
  // array plus the per-segment value streams faster than the table's dependent
  // index loads
  if ((mode == HOP_REAL || mode == HOP_COMPLEX) && n_class <= 4 && !d->no_dictionary) {
    struct Key {
      uint64_t a, b, c;
      int64_t off;
      int32_t cls;
      bool operator==(const Key& o) const {
        return a == o.a && b == o.b && c == o.c && off == o.off && cls == o.cls;
      }
    };
    struct KeyHash {
      size_t operator()(const Key& k) const {
        return std::hash<uint64_t>()(k.a * 0x9E3779B97F4A7C15ull ^ (k.b + 0x632BE59BD9B4E019ull) ^ (k.c << 1) ^
                                     ((uint64_t)k.off * 0xC2B2AE3D27D4EB4Full) ^ ((uint64_t)k.cls << 59));
      }
    };
    auto bits = [](double v) {
      uint64_t u;
      std::memcpy(&u, &v, 8);
      return u;
    };
    std::unordered_map<Key, uint16_t, KeyHash> ids;
    std::vector<double> tab = {0.0, 0.0}, dtab = {0.0};
    std::vector<int32_t> otab = {0}, ctab = {0};
    ids[Key{bits(0.0), bits(0.0), bits(0.0), 0, 0}] = 0;   // padding: offset 0, hopping 0, class 0
    std::vector<uint16_t> hidx(entries, 0);
    bool fits = true;
    for (int64_t sl = 0; sl < n_slices && fits; ++sl) {
      const int64_t w = (slice_ptr[sl + 1] - slice_ptr[sl]) >> S_log2;
      for (int64_t j = 0; j < w && fits; ++j) {
        for (int64_t q = 0; q < S; ++q) {
          const int64_t e = slice_ptr[sl] + j * S + q;
          const int64_t row = sl * S + q;
          if (L->col[e] < 0) continue;
          const double re = mode == HOP_COMPLEX ? L->hop[2 * e] : L->hop[e];
          const double im = mode == HOP_COMPLEX ? L->hop[2 * e + 1] : 0.0;
          const int32_t c = L->cls.empty() ? 0 : L->cls[e];
          const Key key{bits(re), bits(im), bits(L->dx[e]), (int64_t)L->col[e] - row, c};
          auto it = ids.find(key);
          if (it == ids.end()) {
            if ((int64_t)dtab.size() >= kDictMax) {
              fits = false;
              break;
            }
            it = ids.emplace(key, (uint16_t)dtab.size()).first;
            tab.push_back(re);
            tab.push_back(im);
            dtab.push_back(L->dx[e]);
            otab.push_back((int32_t)key.off);
            ctab.push_back(c);
          }
          hidx[e] = it->second;
        }
      }
    }
    if (fits) {
      mode = HOP_DICT;
      L->hidx.swap(hidx);
      L->htab.swap(tab);
      L->dxtab.swap(dtab);
      L->offtab.swap(otab);
      if (!L->cls.empty()) L->cls.swap(ctab);   // classes per table entry from now on
      std::vector<double>().swap(L->hop);
      std::vector<double>().swap(L->dx);
    }
  }

  L->n = n;
  L->n_seg = n_seg;
  L->n_class = n_class;
  L->hop_mode = mode;
  L->S = S;
  L->S_log2 = S_log2;
  L->n_slices = n_slices;
  L->max_width = max_w;
  L->uniform_width = unif_w ? max_deg : 0;
  L->nnz = nnz;
  L->slice_ptr.swap(slice_ptr);
  L->seg_off.swap(seg_off);
  L->seg_dE.swap(dE);
  L->seg_gersh.swap(gersh);
  L->seg_hop.swap(seg_hop);
  return GPUQT_OK;
}

void segment_units(const std::vector<int64_t>& seg_off, std::vector<int64_t>* unit_first,
                   std::vector<int32_t>* starts) {
  const int n_seg = (int)seg_off.size() - 1;
  unit_first->assign(n_seg + 1, 0);
  starts->clear();
  for (int s = 0; s < n_seg; ++s) {
    (*unit_first)[s] = (int64_t)starts->size();
    for (int64_t r = seg_off[s]; r < seg_off[s + 1]; r = ((r >> kUnitLog2) + 1) << kUnitLog2)
      starts->push_back((int32_t)r);
  }
  (*unit_first)[n_seg] = (int64_t)starts->size();
}

void plan_blocks(const std::vector<int64_t>& seg_off, int cus, int per_cu,
                 std::vector<BlkPlan>* plan, std::vector<int32_t>* seg_blk0) {
  const int n_seg = (int)seg_off.size() - 1;
  const int64_t n = seg_off[n_seg];
  const int64_t target = std::max<int64_t>(8, (int64_t)std::max(cus, 1) * std::max(per_cu, 1));
  std::vector<int64_t> unit_first;
  std::vector<int32_t> starts;
  segment_units(seg_off, &unit_first, &starts);
  // workgroups per segment: proportional to rows, at least one, at most one
  // per 64 rows
  std::vector<int64_t> gs(n_seg);
  int64_t G = 0;
  for (int s = 0; s < n_seg; ++s) {
    const int64_t ns = seg_off[s + 1] - seg_off[s];
    int64_t g = (int64_t)std::llround((double)target * (double)ns / (double)n);
    gs[s] = std::max<int64_t>(1, std::min<int64_t>(g, (ns + 63) / 64));
    G += gs[s];
  }
  int64_t padded = G >= 8 ? (G + 7) / 8 * 8 : G;
  gs[n_seg - 1] += padded - G;   // spare workgroups join the last segment
  G = padded;
  const int64_t per_xcd = (G % 8 == 0) ? G / 8 : G;
  plan->assign(G, BlkPlan{0, 0, 0, 1, 0, 0, 0, 0});
  seg_blk0->assign(n_seg + 1, 0);
  int64_t lb = 0;
  for (int s = 0; s < n_seg; ++s) {
    (*seg_blk0)[s] = (int32_t)lb;
    const int64_t a = seg_off[s], b = seg_off[s + 1], ns = b - a;
    const int64_t U = unit_first[s + 1] - unit_first[s];
    // groups: runs of this segment's logical workgroups on one XCD
    std::vector<std::pair<int64_t, int64_t>> groups;   // (first lb, size)
    for (int64_t q = lb; q < lb + gs[s];) {
      const int64_t x = q / per_xcd;
      const int64_t end = std::min(lb + gs[s], (x + 1) * per_xcd);
      groups.push_back({q, end - q});
      q = end;
    }
    // rows of the segment in proportion to group sizes, 64-row aligned; units
    // of a banded order likewise by count
    int64_t done = 0, prev = a, uprev = 0;
    for (size_t k = 0; k < groups.size(); ++k) {
      done += groups[k].second;
      int64_t r = (k + 1 == groups.size()) ? b : a + (ns * done) / gs[s];
      r = std::min(b, std::max(prev, (r / 64) * 64));
      if (k + 1 == groups.size()) r = b;
      // (a multiple of kPencil, so that every group's pencils start aligned)
      const int64_t u = (k + 1 == groups.size()) ? U : std::max(uprev, (U * done) / gs[s] / kPencil * kPencil);
      for (int64_t q = 0; q < groups[k].second; ++q) {
        BlkPlan& P = (*plan)[groups[k].first + q];
        P.r0 = prev;
        P.r1 = r;
        P.j = (int32_t)q;
        P.g = (int32_t)groups[k].second;
        P.seg = s;
        P.u0 = unit_first[s] + uprev;
        P.nu = (int32_t)(u - uprev);
        P.se = b;
      }
      prev = r;
      uprev = u;
    }
    lb += gs[s];
  }
  (*seg_blk0)[n_seg] = (int32_t)G;
}

int64_t row_period(const HostLayout& L, int s) {
  const int64_t a = L.seg_off[s], b = L.seg_off[s + 1];
  if (b <= a) return 0;
  // rows sampled with a stride, enough for a stable 90th percentile
  const int64_t stride = std::max<int64_t>(1, (b - a) / 65536);
  std::vector<int64_t> far;
  far.reserve((size_t)((b - a) / stride + 1));
  for (int64_t r = a; r < b; r += stride) {
    const int64_t sl = r >> L.S_log2;
    const int64_t p0 = L.slice_ptr[sl];
    const int64_t w = (L.slice_ptr[sl + 1] - p0) >> L.S_log2;
    int64_t m = 0;
    for (int64_t j = 0; j < w; ++j) {
      const int32_t c = L.col[p0 + j * L.S + (r & (L.S - 1))];
      if (c >= 0) m = std::max<int64_t>(m, c > r ? c - r : r - c);
    }
    far.push_back(m);
  }
  const size_t k = far.size() / 10;   // 10 % of rows reach less than D
  std::nth_element(far.begin(), far.begin() + k, far.end());
  return far[k];
}

void banded_units(const std::vector<int64_t>& seg_off, const std::vector<int64_t>& period,
                  const std::vector<int64_t>& width, std::vector<int32_t>* out) {
  std::vector<int64_t> unit_first;
  segment_units(seg_off, &unit_first, out);
  const int n_seg = (int)seg_off.size() - 1;
  for (int s = 0; s < n_seg; ++s) {
    const int64_t D = period[s], W = width[s];
    if (W <= 0 || D <= W) continue;   // plain order for this segment
    const int64_t a = seg_off[s];
    auto first = out->begin() + unit_first[s], last = out->begin() + unit_first[s + 1];
    std::stable_sort(first, last, [&](int32_t x, int32_t y) {
      const int64_t ox = x - a, oy = y - a;
      const int64_t bx = (ox % D) / W, by = (oy % D) / W;
      if (bx != by) return bx < by;
      const int64_t qx = ox / D, qy = oy / D;
      if (qx != qy) return qx < qy;
      return ox % D < oy % D;
    });
  }
}

void pencil_units(const std::vector<int64_t>& seg_off, const std::vector<int64_t>& period,
                  const std::vector<int64_t>& width, std::vector<int32_t>* out) {
  std::vector<int64_t> unit_first;
  segment_units(seg_off, &unit_first, out);
  const int n_seg = (int)seg_off.size() - 1;
  for (int s = 0; s < n_seg; ++s) {
    const int64_t D = period[s], W = width[s];
    if (W <= 0 || D < 128) continue;   // plain order for this segment
    const int64_t a = seg_off[s];
    auto first = out->begin() + unit_first[s], last = out->begin() + unit_first[s + 1];
    auto key = [&](int32_t x, int64_t k[5]) {
      const int64_t o = x - a, off = o % D, q = o / D;
      k[0] = off / W;
      k[1] = q / kPencil;
      k[2] = (off % W) >> kUnitLog2;
      k[3] = q % kPencil;
      k[4] = off;
    };
    std::stable_sort(first, last, [&](int32_t x, int32_t y) {
      int64_t kx[5], ky[5];
      key(x, kx);
      key(y, ky);
      for (int i = 0; i < 5; ++i)
        if (kx[i] != ky[i]) return kx[i] < ky[i];
      return false;
    });
  }
}

bool detect_sheets(const gpuqt_h_desc* d, const std::vector<int64_t>& seg_off, std::vector<int32_t>* sheet) {
  sheet->clear();
  if (!d || d->max_nn < 4 || !d->nn || !d->nbr || seg_off.size() < 2) return false;
  const int64_t k = d->max_nn;
  const int n_seg = (int)seg_off.size() - 1;
  std::vector<int32_t> out(2 * (size_t)n_seg);
  for (int sg = 0; sg < n_seg; ++sg) {
    const int64_t a = seg_off[sg], n = seg_off[sg + 1] - a;
    if (n < 9) return false;
    for (int64_t i = a; i < a + n; ++i)
      if (d->nn[i] != 4) return false;
    // the segment's first row (0, 0): its neighbours sorted are 1, Lx - 1, Lx, (Ly - 1) Lx
    int64_t c0[4];
    for (int q = 0; q < 4; ++q) c0[q] = (int64_t)d->nbr[a * k + q] - a;
    std::sort(c0, c0 + 4);
    const int64_t Lx = c0[2];
    if (Lx < 3 || n % Lx != 0) return false;
    const int64_t Ly = n / Lx;
    if (Ly < 3 || n > (int64_t(1) << 24)) return false;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t x = i % Lx, y = i / Lx;
      int64_t e[4] = {(x + 1) % Lx + Lx * y, (x + Lx - 1) % Lx + Lx * y, x + Lx * ((y + 1) % Ly),
                      x + Lx * ((y + Ly - 1) % Ly)};
      int64_t c[4];
      for (int q = 0; q < 4; ++q) c[q] = (int64_t)d->nbr[(a + i) * k + q] - a;
      std::sort(e, e + 4);
      std::sort(c, c + 4);
      for (int q = 0; q < 4; ++q)
        if (c[q] != e[q]) return false;
    }
    out[2 * sg] = (int32_t)Lx;
    out[2 * sg + 1] = (int32_t)Ly;
  }
  *sheet = out;
  return true;
}

int stencil_run(int64_t cols, int len, int64_t workers) {
  workers = std::max<int64_t>(workers, 1);
  int best_z = len;
  int64_t best = -1;
  for (int runs = 1; runs <= len; ++runs) {
    const int z = (len + runs - 1) / runs;
    if (runs > 1 && z < 16) break;
    const int64_t rounds = (cols * ((len + z - 1) / z) + workers - 1) / workers;
    const int64_t cost = rounds * (z + 2);
    if (best < 0 || cost < best) {
      best = cost;
      best_z = z;
    }
  }
  return std::max(best_z, 1);
}

void sheet_split(const std::vector<int64_t>& cols, const std::vector<int32_t>& len, int64_t G,
                 std::vector<int32_t>* blk0, std::vector<int32_t>* zc) {
  const int n = (int)cols.size();
  auto cost = [&](int s, int64_t g) -> int64_t {
    const int z = stencil_run(cols[s], len[s], g);
    const int64_t rounds = (cols[s] * ((len[s] + z - 1) / z) + g - 1) / g;
    return rounds * (z + 2);
  };
  // least workgroups that keep segment s within T (G + 1: none do); cost falls with g
  auto need = [&](int s, int64_t T) -> int64_t {
    if (cost(s, G) > T) return G + 1;
    int64_t lo = 1, hi = G;
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (cost(s, mid) <= T) hi = mid;
      else lo = mid + 1;
    }
    return lo;
  };
  auto fits = [&](int64_t T) {
    int64_t tot = 0;
    for (int s = 0; s < n && tot <= G; ++s) tot += need(s, T);
    return tot <= G;
  };
  int64_t lo = 1, hi = 1;
  for (int s = 0; s < n; ++s) hi = std::max(hi, cost(s, 1));
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (fits(mid)) hi = mid;
    else lo = mid + 1;
  }
  std::vector<int64_t> g(n);
  int64_t used = 0;
  int big = 0;
  for (int s = 0; s < n; ++s) {
    g[s] = std::max<int64_t>(1, need(s, lo));
    used += g[s];
    if (cols[s] * len[s] > cols[big] * len[big]) big = s;
  }
  g[big] += G - used;
  blk0->assign(n + 1, 0);
  zc->assign(n, 1);
  for (int s = 0; s < n; ++s) {
    (*blk0)[s + 1] = (*blk0)[s] + (int32_t)g[s];
    (*zc)[s] = stencil_run(cols[s], len[s], g[s]);
  }
}

bool detect_box(const gpuqt_h_desc* d, int32_t box[3]) {
  box[0] = box[1] = box[2] = 0;
  if (!d || d->n < 27 || d->max_nn < 6 || (d->n_segments > 1) || !d->nn || !d->nbr) return false;
  const int64_t n = d->n;
  const int64_t k = d->max_nn;
  for (int64_t i = 0; i < n; ++i)
    if (d->nn[i] != 6) return false;
  // row 0 = (0, 0, 0): its neighbours sorted are 1, Lx - 1, Lx, (Ly - 1) Lx, Lx Ly, (Lz - 1) Lx Ly
  int64_t c0[6];
  for (int s = 0; s < 6; ++s) c0[s] = d->nbr[s];
  std::sort(c0, c0 + 6);
  const int64_t Lx = c0[2], LxLy = c0[4];
  if (Lx < 3 || LxLy % Lx != 0) return false;
  const int64_t Ly = LxLy / Lx;
  if (Ly < 3 || n % LxLy != 0) return false;
  const int64_t Lz = n / LxLy;
  if (Lz < 3 || Lx > INT32_MAX || Ly > INT32_MAX || Lz > INT32_MAX) return false;
  // the box kernels address a plane of a block with 32-bit byte offsets: a plane of 16
  // vectors of 16-byte elements must span at most 4 GiB
  if (LxLy > (int64_t(1) << 24)) return false;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t x = i % Lx, y = (i / Lx) % Ly, z = i / LxLy;
    int64_t e[6] = {(x + 1) % Lx + Lx * (y + Ly * z),      (x + Lx - 1) % Lx + Lx * (y + Ly * z),
                    x + Lx * ((y + 1) % Ly + Ly * z),      x + Lx * ((y + Ly - 1) % Ly + Ly * z),
                    x + Lx * (y + Ly * ((z + 1) % Lz)),    x + Lx * (y + Ly * ((z + Lz - 1) % Lz))};
    int64_t c[6];
    for (int s = 0; s < 6; ++s) c[s] = d->nbr[i * k + s];
    std::sort(e, e + 6);
    std::sort(c, c + 6);
    for (int s = 0; s < 6; ++s)
      if (c[s] != e[s]) return false;
  }
  box[0] = (int32_t)Lx;
  box[1] = (int32_t)Ly;
  box[2] = (int32_t)Lz;
  return true;
}

bool box_dx_uniform(const HostLayout& L, const int32_t box[3], double* dx) {
  const int64_t Lx = box[0], Ly = box[1], LxLy = (int64_t)box[0] * box[1];
  if (Lx <= 0 || L.uniform_width != 6 || L.dx.empty() || L.col.empty()) return false;
  const int S = L.S;
  double delta = 0.0;
  bool have = false;
  for (int64_t r = 0; r < L.n; ++r) {
    const int64_t x = r % Lx, yz = r / Lx;
    const int64_t xp = (x + 1) % Lx + Lx * yz, xm = (x + Lx - 1) % Lx + Lx * yz;
    const int64_t base = (r / S) * (int64_t)(6 * S) + (r % S);
    for (int j = 0; j < 6; ++j) {
      const int64_t e = base + (int64_t)j * S;
      const int64_t c = L.col[e];
      const double d = L.dx[e];
      if (c == xp) {
        if (!have) {
          delta = d;
          have = true;
        }
        if (d != delta) return false;
      } else if (c == xm) {
        if (!have) {
          delta = -d;
          have = true;
        }
        if (d != -delta) return false;
      } else if (d != 0.0) {
        return false;
      }
    }
  }
  (void)Ly;
  (void)LxLy;
  if (!have) return false;
  *dx = delta;
  return true;
}

}  // namespace gpuqt
