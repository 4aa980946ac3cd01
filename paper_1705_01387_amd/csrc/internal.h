// Internal declarations shared by the host API (api.cpp, layout.cpp) and the
// HIP kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gpuqt.h"

namespace gpuqt {

// Hopping storage: one value per segment, a double or a complex double per
// entry, or (HOP_DICT) a 16-bit index per entry into a table of the distinct
// (column offset, hopping, position difference) triples, which then replaces
// the column indices too.
enum HopMode { HOP_UNIFORM = 0, HOP_REAL = 1, HOP_COMPLEX = 2, HOP_DICT = 3 };
constexpr int kDictMax = 65535;     // table entries of HOP_DICT (index 0: padding, value 0)

constexpr int kBlock = 256;         // threads per workgroup of every sparse kernel
constexpr int kPerCU = 8;           // resident workgroups per CU of the primary plan
// Hot kernel families; each launches with the plan whose workgroup count its
// compiled occupancy keeps resident all at once (a grid larger than what fits
// would leave a tail of workgroups that start only when others finish).
enum Family {
  FAM_MOMENT = 0, FAM_SYM = 1, FAM_PAIR = 2, FAM_EVOLVE = 3, FAM_MSD = 4, FAM_EVOLVE_PAIR = 5, kFamilies = 6
};
constexpr int kRowAlign = 256;      // block row ranges start at multiples of this
constexpr int kMaxB = 16;           // widest vector block

// Rows of one logical workgroup.  The workgroup is member j of a group of g
// workgroups of segment seg; it visits the tiles j, j + g, j + 2g, ... of
// the group's row sequence, which is either
//   linear: the contiguous rows [r0, r1), or
//   banded: the 64-row units units[u0 .. u0 + nu) of a banded unit order
//           (each unit is the part of one 64-row slice inside the segment,
//           whose rows end at se), or of a pencil order (see row_at_pencil).
struct BlkPlan {
  int64_t r0, r1;
  int32_t j, g, seg, nu;
  int64_t u0, se;
};

constexpr int kUnitLog2 = 6;        // rows per unit of a banded order: 64
constexpr int kPencil = kBlock / 64;   // units per pencil: one per wavefront of a workgroup
constexpr int kSheetCells = 1;      // cells per lane of a sheet kernel strip (kSheetCells * 256 / B cells)
constexpr int kTuneTimes = 7;       // entries of gpuqt_autotune's times_us: 4 load/order variants, 2 pencil, box
constexpr int kNumB = 5;            // block widths 1, 2, 4, 8, 16
constexpr int64_t kBandBudget = int64_t(5) << 19;   // 2.5 MiB: bytes one row window may stream per XCD

#if defined(__HIPCC__)
#define GPUQT_PLAN_HD __host__ __device__
#else
#define GPUQT_PLAN_HD
#endif

// Row at position pos of a workgroup's row sequence, or -1 for an idle lane
// (past the end of a clipped unit).  pos < row_seq_len(P, units).
//   linear: r0 + pos;  banded: the pos % 64-th row of unit pos / 64.
GPUQT_PLAN_HD inline int64_t row_seq_len(const BlkPlan& P, const int32_t* units) {
  return units ? ((int64_t)P.nu << kUnitLog2) : (P.r1 - P.r0);
}
GPUQT_PLAN_HD inline int64_t row_at(const BlkPlan& P, const int32_t* units, int64_t pos) {
  if (!units) return P.r0 + pos;
  const int64_t a = units[P.u0 + (pos >> kUnitLog2)];
  const int64_t r = a + (pos & ((int64_t(1) << kUnitLog2) - 1));
  const int64_t end = ((a >> kUnitLog2) + 1) << kUnitLog2;
  return (r < end && r < P.se) ? r : -1;
}

// Pencil order: the group's units are taken kPencil at a time, one per
// wavefront.  Tile t (of kBlock / B rows) covers rows sub * RPW .. sub * RPW +
// RPW - 1 of units kPencil * (t / B) + w (wavefront w), sub = t mod B, RPW =
// 64 / B rows per wavefront, so the wavefronts of one workgroup (one CU and its
// L1) work on the same rows of kPencil units at once: in a pencil unit order
// those are units one lattice period apart, whose rows gather each other.
// The sequence has kPencil * 64 * ceil(nu / kPencil) positions.
GPUQT_PLAN_HD inline int64_t pencil_seq_len(const BlkPlan& P) {
  return (int64_t)((P.nu + kPencil - 1) / kPencil) * kPencil << kUnitLog2;
}
GPUQT_PLAN_HD inline int64_t row_at_pencil(const BlkPlan& P, const int32_t* units, int64_t pos, int B) {
  const int rpi = kBlock / B, rpw = 64 / B;
  const int64_t t = pos / rpi;
  const int q = (int)(pos % rpi);
  const int64_t u = (t / B) * kPencil + q / rpw;
  if (u >= P.nu) return -1;
  const int64_t a = units[P.u0 + u];
  const int64_t r = a + (t % B) * rpw + q % rpw;
  const int64_t end = ((a >> kUnitLog2) + 1) << kUnitLog2;
  return (r < end && r < P.se) ? r : -1;
}

// Device view of a Hamiltonian in sliced ELL.  Rows are cut into slices of S
// rows; slice s stores width_s entries per row, slot-major (entry j of row
// s*S + r sits at slice_ptr[s] + j*S + r), so a wavefront reading one slot of
// consecutive rows reads consecutive addresses.  Missing neighbours are
// padding entries with col = -1.  Hoppings and on-site terms are stored
// already divided by the segment's DeltaE (H~ = H / DeltaE, Section 3.2).
struct DevMat {
  const int64_t* slice_ptr;  // [n_slices + 1] first entry of each slice
  const int32_t* col;        // [entries] neighbour index or -1
  const double* hop;         // HOP_REAL: [entries]; HOP_COMPLEX: [2*entries] (re, im)
  const double* dx;          // [entries] x_col - x_row (minimum image), 0 for padding (not HOP_DICT)
  const uint16_t* hidx;      // HOP_DICT: [entries] table index of each entry
  const double2* htab;       // HOP_DICT: [T] hopping of each table entry (re, im)
  const double* dxtab;       // HOP_DICT: [T] position difference of each table entry
  const int32_t* offtab;     // HOP_DICT: [T] column offset (column - row) of each table entry
  const double* diag;        // [n] U_i / DeltaE_seg
  const BlkPlan* plan;       // [G] row ranges of the logical workgroups
  const int32_t* units;      // banded or pencil unit order for this block width (first row of each unit), or NULL
  int32_t pencil;            // 1: units is a pencil order, visited as row_at_pencil says
  int32_t box[3];            // (Lx, Ly, Lz) of a periodic box stencil the Hermitian step may use, else 0
  int32_t use_box;           // 1: the Hermitian step runs the box stencil kernel
  int32_t use_box_msd;       // 1: the MSD term runs the box stencil kernel (box_dx valid)
  double box_dx;             // x_{i+1} - x_i of the box's x neighbours (the only non-zero dx)
  int32_t use_sheet;         // 1: the Hermitian step runs the sheet stencil kernel
  int32_t sheet_nseg;        // segments of the sheet tables
  const int32_t* sheet;      // [2 n_seg] (Lx, Ly) of each segment when all are periodic squares
  const int64_t* sheet_off;  // [n_seg] first row of each segment
  const int32_t* sheet_zc;   // [n_seg] rows per work item of the sheet kernel at this plan and B
  const int32_t* sheet_blk0; // [n_seg + 1] first logical workgroup of each segment in the sheet
                             // kernel's own split of this plan's workgroups at this B
  const double* seg_dE;      // [n_seg] DeltaE of each segment
  const double* seg_hop;     // [n_seg] uniform hopping / DeltaE (HOP_UNIFORM)
  // the hoppings given at build time (before class scales), for class gradients
  // dL/ds_c: hop0 like hop, htab0 like htab, seg_hop0 like seg_hop
  const double* hop0;
  const double2* htab0;
  const double* seg_hop0;
  int64_t n;
  int32_t S_log2;
  int32_t G;
  int32_t K;                 // entries per row when every slice has the same width, else 0
  int32_t nt;                // 1: non-temporal loads for the once-read streams (host dispatch)
};

struct Handle {
  int device = 0;
  int64_t n = 0;
  int32_t n_seg = 1;
  int32_t n_class = 1;
  int32_t hop_mode = HOP_REAL;
  int32_t S = 64;
  int32_t S_log2 = 6;
  int64_t n_slices = 0;
  int64_t entries = 0;
  int64_t nnz = 0;
  int32_t max_width = 0;
  int32_t uniform_width = 0;
  int32_t G = 0;
  size_t device_bytes = 0;
  std::vector<int64_t> seg_off;   // host copy [n_seg + 1]
  std::vector<double> seg_dE;     // host copy
  std::vector<double> seg_gersh;  // host copy
  std::vector<BlkPlan> plan_host;
  int32_t nt = 1;                 // kernel variant chosen by gpuqt_autotune (or the default)
  // plans for p = 1 .. kPerCU resident workgroups per CU (index p - 1; the last is
  // the primary plan d_plan / d_seg_blk0 / G)
  BlkPlan* d_plans[kPerCU] = {};
  int32_t* d_blk0s[kPerCU] = {};
  int32_t Gs[kPerCU] = {};
  // resident workgroups per CU of each hot family [family][log2 B][nt] (0: unknown)
  int8_t occ[kFamilies][kNumB][2] = {};
  int32_t banded = 0;             // 1: use the banded unit order where one exists
  int32_t pencil = 0;             // with banded: the pencil unit order instead, where one exists
  // 1: the series families (evolution terms, MSD term) use the other load variant
  // (non-temporal <-> plain) than nt
  int32_t series_nt_flip = 0;
  // periodic box of the matrix (detect_box), and whether the Hermitian step of blocks of
  // B >= 2 vectors uses the box stencil kernel for it
  int32_t box[3] = {0, 0, 0};
  int32_t use_box = 0;
  // the box's position differences: 0 for the y and z neighbours and +-box_dx for the x
  // neighbours on every row (box_msd_ok), which the MSD term's box kernel needs
  int32_t box_msd_ok = 0;
  double box_dx = 0.0;
  int32_t use_box_msd = 0;
  // every segment a periodic square (detect_sheets): d_sheet [2 n_seg] = (Lx, Ly),
  // d_sheet_off [n_seg] their first rows, and per plan and block width the sheet kernel's
  // split of the plan's workgroups over the segments (sheet_split),
  // d_sheet_blk0[(plan * kNumB + log2 B) * (n_seg + 1) + s], and its rows per work item,
  // d_sheet_zc[(plan * kNumB + log2 B) * n_seg + s]; use_box selects the sheet kernel too
  int32_t sheet_ok = 0;
  int32_t* d_sheet = nullptr;
  int64_t* d_sheet_off = nullptr;
  int32_t* d_sheet_zc = nullptr;
  int32_t* d_sheet_blk0 = nullptr;
  bool sheet_in_use(int B) const { return sheet_ok && use_box && B >= 2 && hop_mode == HOP_UNIFORM; }
  // at most this many resident workgroups per CU (0: as many as fit).  Fewer
  // waves in flight can beat full occupancy when the gathers reuse cached
  // lines: the window of rows in flight, and so the cache footprint, shrinks.
  int32_t per_cu_cap = 0;
  // per kernel family: -1 = use per_cu_cap, else that family's own cap (0: none)
  int8_t fam_cap[kFamilies] = {-1, -1, -1, -1, -1, -1};
  // banded orders per block width (index log2 B); NULL where the plain row order
  // already keeps the neighbour window within the cache budget
  int32_t* d_units[kNumB] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  // pencil orders per block width; NULL where no segment has a period of at least 128 rows
  int32_t* d_units_p[kNumB] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int32_t pencil_rows[kNumB] = {0, 0, 0, 0, 0};
  std::vector<int64_t> seg_period;   // detected row period D per segment (0: none)
  int32_t band_rows[kNumB] = {0, 0, 0, 0, 0};
  // device allocations
  int64_t* d_slice_ptr = nullptr;
  int32_t* d_col = nullptr;
  double* d_hop = nullptr;
  double* d_dx = nullptr;
  uint16_t* d_hidx = nullptr;      // HOP_DICT
  double* d_htab = nullptr;        // HOP_DICT [2T]
  double* d_htab0 = nullptr;       // HOP_DICT: build-time table (allocated on the first class update)
  double* d_dxtab = nullptr;       // HOP_DICT [T]
  int32_t* d_offtab = nullptr;     // HOP_DICT [T]
  int32_t dict_size = 0;
  int32_t max_nn_in = 0;           // neighbour slots per orbital of the descriptor (per-entry gradients)
  double* d_diag = nullptr;
  int32_t* d_cls = nullptr;
  BlkPlan* d_plan = nullptr;
  int32_t* d_seg_blk0 = nullptr;   // [n_seg + 1] first logical workgroup of each segment
  double* d_seg_dE = nullptr;
  double* d_seg_hop = nullptr;
  double* d_seg_hop0 = nullptr;    // [n_seg] build-time uniform hopping / DeltaE
  // parameter updates: build-time hoppings (allocated on the first class update),
  // current class scales, per-workgroup spectrum bounds
  double* d_hop0 = nullptr;
  double* d_bound = nullptr;
  std::vector<double> seg_hop0;
  std::vector<double> class_scale;
  // opt-in timing (gpuqt_set_timing): event pairs around runs of one kernel family
  struct TimingRec {
    int family;
    hipEvent_t a, b;
    int64_t launches;
  };
  bool timing = false;
  mutable std::vector<TimingRec> timing_recs;

  static int log2B(int B) { return B <= 1 ? 0 : B == 2 ? 1 : B == 4 ? 2 : B == 8 ? 3 : 4; }

  // plan of a hot family at block width B and the current load variant
  // load variant of a kernel family
  int fam_nt(int family) const {
    const bool series = family == FAM_EVOLVE || family == FAM_EVOLVE_PAIR || family == FAM_MSD;
    return series ? (nt ^ series_nt_flip) : nt;
  }
  int plan_index(int B, int family) const {
    int p = occ[family][log2B(B)][fam_nt(family) ? 1 : 0];
    if (p < 1 || p > kPerCU) p = kPerCU;
    const int cap = fam_cap[family] >= 0 ? fam_cap[family] : per_cu_cap;
    if (cap > 0 && cap < p) p = cap;
    return p - 1;
  }
  // per family f, bits 3f..3f+2: fam_cap[f] + 1 (0: the handle's cap; family caps are 0..6)
  int32_t family_caps_code() const {
    int32_t c = 0;
    for (int f = 0; f < kFamilies; ++f) c |= (int32_t)(fam_cap[f] + 1) << (3 * f);
    return c;
  }
  // nt | banded << 1 | per_cu_cap << 2 | pencil << 6 | series_nt_flip << 7 | (fam_cap[f] + 1) << (8 + 3 f)
  // | use_box << 26 | use_box_msd << 27
  int32_t variant_code() const {
    return nt | (banded << 1) | (per_cu_cap << 2) | ((banded & pencil) << 6) | (series_nt_flip << 7) |
           (family_caps_code() << 8) | ((box[0] > 0 || sheet_ok ? use_box : 0) << 26) |
           ((box_msd_ok ? use_box_msd : 0) << 27);
  }
  int G_of(int B, int family) const { return Gs[plan_index(B, family)]; }
  // first logical workgroup of each segment for the reduction of a family's partials: the
  // plan's, or for the Hermitian step on sheets the sheet kernel's own split
  const int32_t* blk0_of(int B, int family) const {
    const int i = plan_index(B, family);
    if (family == FAM_SYM && sheet_in_use(B)) return d_sheet_blk0 + ((int64_t)i * kNumB + log2B(B)) * (n_seg + 1);
    return d_blk0s[i];
  }
  DevMat view(int B, int family) const {
    DevMat m = view(B);
    const int i = plan_index(B, family);
    m.plan = d_plans[i];
    m.G = Gs[i];
    m.nt = fam_nt(family);
    m.sheet_zc = d_sheet_zc ? d_sheet_zc + ((int64_t)i * kNumB + log2B(B)) * n_seg : nullptr;
    m.sheet_blk0 = d_sheet_blk0 ? d_sheet_blk0 + ((int64_t)i * kNumB + log2B(B)) * (n_seg + 1) : nullptr;
    return m;
  }

  DevMat view(int B) const {
    DevMat m;
    const int lb = log2B(B);
    m.pencil = (banded && pencil && d_units_p[lb]) ? 1 : 0;
    m.units = m.pencil ? d_units_p[lb] : (banded ? d_units[lb] : nullptr);
    m.box[0] = box[0];
    m.box[1] = box[1];
    m.box[2] = box[2];
    m.use_box = (box[0] > 0 && use_box) ? 1 : 0;
    m.use_box_msd = (box[0] > 0 && box_msd_ok && use_box_msd) ? 1 : 0;
    m.box_dx = box_dx;
    m.use_sheet = (sheet_ok && use_box) ? 1 : 0;
    m.sheet = d_sheet;
    m.sheet_off = d_sheet_off;
    m.sheet_nseg = n_seg;
    m.sheet_zc = d_sheet_zc ? d_sheet_zc + ((int64_t)(kPerCU - 1) * kNumB + lb) * n_seg : nullptr;
    m.sheet_blk0 = d_sheet_blk0 ? d_sheet_blk0 + ((int64_t)(kPerCU - 1) * kNumB + lb) * (n_seg + 1) : nullptr;
    m.slice_ptr = d_slice_ptr;
    m.col = d_col;
    m.hop = d_hop;
    m.dx = d_dx;
    m.hidx = d_hidx;
    m.htab = reinterpret_cast<const double2*>(d_htab);
    m.dxtab = d_dxtab;
    m.offtab = d_offtab;
    m.diag = d_diag;
    m.plan = d_plan;
    m.seg_dE = d_seg_dE;
    m.seg_hop = d_seg_hop;
    m.hop0 = d_hop0 ? d_hop0 : d_hop;
    m.htab0 = reinterpret_cast<const double2*>(d_htab0 ? d_htab0 : d_htab);
    m.seg_hop0 = d_seg_hop0;
    m.n = n;
    m.S_log2 = S_log2;
    m.G = G;
    m.K = uniform_width;
    m.nt = nt;
    return m;
  }
};

// Host-side layout produced by layout.cpp from a descriptor (pure C++).
struct HostLayout {
  int64_t n = 0;
  int32_t n_seg = 1;
  int32_t n_class = 1;
  int32_t hop_mode = HOP_REAL;
  int32_t S = 64;
  int32_t S_log2 = 6;
  int64_t n_slices = 0;
  int32_t max_width = 0;
  int32_t uniform_width = 0;
  int64_t nnz = 0;
  std::vector<int64_t> slice_ptr;
  std::vector<int32_t> col;
  std::vector<double> hop;   // real or interleaved complex, or empty (uniform)
  std::vector<double> dx;
  std::vector<uint16_t> hidx;  // HOP_DICT
  std::vector<double> htab;    // HOP_DICT, interleaved (re, im)
  std::vector<double> dxtab;   // HOP_DICT
  std::vector<int32_t> offtab; // HOP_DICT
  std::vector<double> diag;
  std::vector<int32_t> cls;  // class per entry, -1 for padding (per table entry in HOP_DICT; empty if one class)
  std::vector<int64_t> seg_off;
  std::vector<double> seg_dE;
  std::vector<double> seg_gersh;
  std::vector<double> seg_hop;
};

// Set the calling thread's gpuqt_last_error text and return st (api.cpp).
gpuqt_status set_error(gpuqt_status st, const std::string& msg);

// layout.cpp: validate the descriptor and build the sliced ELL on the host.
// Returns GPUQT_OK or an error status with *msg set.
gpuqt_status build_host_layout(const gpuqt_h_desc* d, HostLayout* L, std::string* msg);

// Workgroup plan: about `per_cu` resident workgroups per compute unit, split
// over the segments in proportion to their rows; G is a multiple of 8 when
// G >= 8 (logical workgroup x*G/8 .. (x+1)*G/8-1 run on XCD x).  The logical
// workgroups of one segment on one XCD form a group over a contiguous,
// 64-row aligned part of the segment, and over a contiguous part of the
// segment's units in a banded order (the same count split for every order).
// seg_blk0[s] is the first logical workgroup of segment s (seg_blk0[n_seg] = G).
void plan_blocks(const std::vector<int64_t>& seg_off, int cus, int per_cu,
                 std::vector<BlkPlan>* plan, std::vector<int32_t>* seg_blk0);

// Units (64-row slices clipped to segments) of every segment, in segment order:
// unit_first[s] is the index of segment s's first unit, starts[u] its first row.
void segment_units(const std::vector<int64_t>& seg_off, std::vector<int64_t>* unit_first,
                   std::vector<int32_t>* starts);

// Row period D of a segment: the neighbour offset |c - r| that 90 % of rows
// reach or exceed as their largest one (in a lattice numbered lexicographically,
// the stride of its slowest index).  0 when the segment has no off-diagonal entries.
int64_t row_period(const HostLayout& L, int s);

// Banded order of the units of each segment for band width W rows: unit at
// offset a from the segment start goes to (band (a mod D) / W, sweep a / D,
// a mod D), so rows one period apart are visited W rows apart instead of D.
// W is given per segment (width[s]); segments with W = 0, D = 0 or D <= W keep
// the plain order.
void banded_units(const std::vector<int64_t>& seg_off, const std::vector<int64_t>& period,
                  const std::vector<int64_t>& width, std::vector<int32_t>* out);

// Pencil order of the units of each segment for band width W rows: unit at
// offset a goes to (band (a mod D) / W, sweep group (a / D) / kPencil, 64-row
// bucket of (a mod D) within the band, sweep (a / D) mod kPencil, a mod D), so
// kPencil consecutive units are the same rows of kPencil consecutive periods
// (as far as the 64-row units line up with the period).  Segments with W = 0 or
// D < 128 keep the plain order.
void pencil_units(const std::vector<int64_t>& seg_off, const std::vector<int64_t>& period,
                  const std::vector<int64_t>& width, std::vector<int32_t>* out);

// A periodic simple cubic box in natural order: one segment, every row i = x + Lx (y + Ly z)
// with exactly the six neighbours (x +- 1 mod Lx, y, z), (x, y +- 1 mod Ly, z),
// (x, y, z +- 1 mod Lz) in any slot order, Lx, Ly, Lz >= 3 and Lx Ly <= 2^24 (so that a
// plane of a block of up to 16 vectors spans at most 4 GiB).  box = (Lx, Ly, Lz) when it
// is one (checked row by row), else (0, 0, 0).
bool detect_box(const gpuqt_h_desc* d, int32_t box[3]);

// The position differences of a detected box in layout L (uniform width 6): true, with
// *dx = x_{i+1} - x_i, when every row's x neighbours have dx = +dx and -dx and its y and z
// neighbours dx = 0.
bool box_dx_uniform(const HostLayout& L, const int32_t box[3], double* dx);

// Every segment s of layout L (rows seg_off[s] ..) a periodic Lx x Ly square in natural
// order: row seg_off[s] + x + Lx y with exactly the four neighbours (x +- 1 mod Lx, y) and
// (x, y +- 1 mod Ly) in any slot order, Lx, Ly >= 3, Lx Ly <= 2^24 (a segment of a block
// of 16 vectors spans at most 4 GiB: the sheet kernel addresses it with 32-bit offsets).
// sheet = (Lx, Ly) per segment when all are, else false.
bool detect_sheets(const gpuqt_h_desc* d, const std::vector<int64_t>& seg_off, std::vector<int32_t>* sheet);

// Length of a run of a stencil kernel's march: cols columns (or strips) of work items
// over len planes (or rows), shared by `workers` workgroups that take the items in turn.
// A run of z steps costs a workgroup z + 2 loads of its column (the steps before and after
// the run come again) and the items go round in ceil(cols * runs / workers) rounds: the
// run length that minimises rounds * (z + 2), at least 16 unless one run covers len.
int stencil_run(int64_t cols, int len, int64_t workers);

// The sheet kernel's split of G workgroups over segments of cols[s] strips and len[s] rows:
// the fewest workgroups per segment that keep every segment's longest chain (stencil_run's
// rounds * (z + 2)) within a common bound, the least bound the G workgroups allow (found
// by bisection); workgroups left over join the segment of most work.  blk0[s] = first
// workgroup of segment s (blk0[n] = G), zc[s] = its rows per work item.  Needs G >= n.
void sheet_split(const std::vector<int64_t>& cols, const std::vector<int32_t>& len, int64_t G,
                 std::vector<int32_t>* blk0, std::vector<int32_t>* zc);

// Running conductivity over time rows (mode 0: VAC integral, 1: MSD derivative).
// Transport quantities of Section 2.2 from reconstructed rows (see gpuqt_transport_lengths).
struct TransportIO {
  int n_t, n_E;
  const double* rho;     // [n_E]
  const double* vac0;    // [n_E] rho C_vv at t = 0, or NULL
  const double* sigma;   // [n_t][n_E] running conductivity, or NULL
  const double* msd;     // [n_t][n_E] rho DeltaX^2, or NULL
  double *sigma_sc, *v, *tau, *mfp, *xi;   // [n_E] each, or NULL
  double* L;             // [n_t][n_E], or NULL
};
hipError_t launch_transport(const TransportIO& io, hipStream_t s);

hipError_t launch_sigma(int mode, int n_t, const double* dt, int n_E, const double* y, double* out,
                        hipStream_t s);

// Resident workgroups per CU of a hot family's kernel for this layout (hopping
// mode, row width A.K), block width B and load variant nt (kernels.hip).
int kernel_occupancy(int family, const DevMat& A, int hop_mode, int B, int nt);

// ----------------------------------------------------------------------------
// Kernel launchers (kernels.hip).  All return hipSuccess or the launch error.
// Vectors are double2 [n][B].
// ----------------------------------------------------------------------------
struct StepIO {
  const double2* x;    // gathered input (v_{n-1})
  const double2* w;    // v_{n-2} (unused when first)
  double2* out;        // v_n
  int first;           // 1: v_1 = H~ v_0 (no factor 2, no subtraction)
};

// One Chebyshev moment step: out = 2 H~ x - w (or H~ x), and per-workgroup
// partial sums of <phiL|out> into part_n[lb*B + b] (and <phiL|x> into part_0
// when first).
hipError_t launch_moment_step(const DevMat& A, int hop_mode, int B, const StepIO& io,
                              const double2* phiL, double2* part_n, double2* part_0,
                              hipStream_t s);

// One term of the evolution series: a_m as in a moment step, and
// acc += c_m a_m with c_m = J[seg*ldJ + m] * phase (first: acc = c_0 a_0 + c_1 a_1).
hipError_t launch_evolve_term(const DevMat& A, int hop_mode, int B, const StepIO& io,
                              double2* acc, const double* Jtab, int ldJ, int m, double2 phase_m,
                              double2 phase_0, hipStream_t s);

// One term of the fused evolution + commutator series (a- and b-chains).
struct ChainIO {
  const double2* xa; const double2* wa; double2* oa;   // a-chain: T_m psi
  const double2* xb; const double2* wb; double2* ob;   // b-chain: [X,T_m] psi + T_m chi
  int first;
  int has_b0;                                          // b_0 = chi_in is non-zero
};
hipError_t launch_msd_term(const DevMat& A, int hop_mode, int B, const ChainIO& io,
                           double2* acc_a, double2* acc_b, const double* Jtab, int ldJ, int m,
                           double2 phase_m, double2 phase_0, hipStream_t s);

// One term of U(dt) on two vectors (chains a and b of io, has_b0 unused):
// acc_a += c_m a_m, acc_b += c_m b_m.
hipError_t launch_evolve_pair_term(const DevMat& A, int hop_mode, int B, const ChainIO& io, double2* acc_a,
                                   double2* acc_b, const double* Jtab, int ldJ, int m, double2 phase_m,
                                   double2 phase_0, hipStream_t s);

// out = V x (which = GPUQT_VELOCITY) or [X,H] x (GPUQT_COMMUTATOR_XH), unscaled H;
// with kAccumulate or-ed into `which`, out += instead.
constexpr int kAccumulate = 2;
hipError_t launch_commutator(const DevMat& A, int hop_mode, int B, int which, const double2* x,
                             double2* out, hipStream_t s);

// out = J_0 * in (Np = 1 evolution), per segment.
hipError_t launch_scale(const DevMat& A, int B, const double2* in, double2* out,
                        const double* Jtab, int ldJ, hipStream_t s);

// One reverse step of the moment recurrence (kernels_adjoint.hip):
//   out = wts[seg][b][n] * phiL + f_rec * H~ x - w    (x, w may be NULL: zero)
// and, when v (= v_{n-1}) is given, gU[r] += f sum_b Re(conj(out) v) / DeltaE and
// gcp[lb][c] += f Re <out| H~_c v> over the workgroup's rows.
struct AdjIO {
  const double2* x;      // lam_{n+1}, gathered
  const double2* w;      // lam_{n+2}
  double2* out;          // lam_n
  const double2* phiL;
  const double* wts;     // [n_seg][B][M] loss weights on Re mu (NULL: zero)
  int32_t M, n;
  double f_rec;          // 2 for a reverse step, 1 for lam_0
  const double2* v;      // v_{n-1} (NULL: no gradient terms)
  double f;              // 2 for n >= 2, 1 for n = 1
  double* gU;            // [n] accumulated
  double* gcp;           // [G][nc] accumulated per workgroup
  const int32_t* cls;    // class of each entry, or (HOP_DICT) of each table entry (nc > 1)
  const double* Jtab;    // non-NULL: source coefficient J[seg*ldJ + n] * src_phase instead of wts
  int32_t ldJ;
  int32_t accumulate;    // 1: out += lam (instead of out = lam)
  double2 src_phase;
  double* gH;            // NULL, or per-entry gradients [n][ldH] (re, im) pairs, accumulated
  int32_t ldH;           // entry slots per row of gH (the descriptor's max_nn)
};
// Reverse of the two-chain (product identity) moment computation: chains
// a_k = T_k a_0, b_k = T_k b_0 and L = sum_n om_n Re r_n over the raw dots
// r_2k = <a_k|b_k>, r_2k-1 = <a_k|b_k-1>, r_0 = <a_0|b_0>; one step k yields
// abar_k = om_2k b_k + om_2k-1 b_k-1 + f_rec H~ abar_k+1 - abar_k+2 and
// bbar_k = om_2k a_k + om_2k+1 a_k+1 + f_rec H~ bbar_k+1 - bbar_k+2.
struct AdjPairIO {
  const double2* xa;     // abar_{k+1}, gathered (NULL: zero)
  const double2* wa;     // abar_{k+2} (NULL: zero)
  double2* oa;           // abar_k
  const double2* xb;
  const double2* wb;
  double2* ob;
  const double2* a_m1;   // a_{k-1} (gradient terms; NULL for k = 0)
  const double2* a_k;
  const double2* a_p1;   // a_{k+1} (NULL: om_{2k+1} = 0)
  const double2* b_m1;
  const double2* b_k;
  const double* om;      // [n_seg][B][R] raw-dot weights
  int32_t R, k;
  double f_rec;          // 2 for k >= 1, 1 for k = 0
  double f;              // gradient factor: 2 for k >= 2, 1 for k = 1 (unused for k = 0)
  double* gU;            // [n] accumulated (NULL: no parameter terms)
  double* gcp;           // [G][nc] accumulated per workgroup
  const int32_t* cls;
  int32_t acc_a, acc_b;  // 1: oa += abar_k, ob += bbar_k
};
hipError_t launch_adjoint_pair_step(const DevMat& A, int hop_mode, int B, int nc, const AdjPairIO& io,
                                    hipStream_t s);
// om[s][b][r] for r < R from loss weights w[s][b][n], n < M (raw-dot weights of
// the product identities: om_0 = w_0 - sum of even w_n (n >= 2), om_1 = w_1 -
// sum of odd w_n (n >= 3), om_n = 2 w_n for 2 <= n < M, 0 beyond)
hipError_t launch_raw_weights(const double* w, int rows, int M, int R, double* om, hipStream_t s);

// parameter updates (gpuqt_update_h_values)
constexpr int kMaxUpdateClasses = 8;
struct ClassScale {
  double s[kMaxUpdateClasses];
};
hipError_t launch_set_onsite(const DevMat& A, const double* onsite, double* diag, hipStream_t s);
hipError_t launch_scale_hops(int64_t entries, int cplx, const double* hop0, double* hop,
                             const int32_t* cls, const ClassScale& sc, hipStream_t s);
// bound[lb] = max over rows of |U~_r| + sum_j |H~_rj|
hipError_t launch_row_bound(const DevMat& A, int hop_mode, double* bound, hipStream_t s);

// gcp[lb][c] += Re sum_i conj(a_i) (V_c x)_i, V_c = i dx H_c (unscaled)
hipError_t launch_velocity_class_grad(const DevMat& A, int hop_mode, int B, int nc, const double2* a,
                                      const double2* x, const int32_t* cls, double* gcp, hipStream_t s);
// per-entry share of the velocity V = i dx H (unscaled): g_ij = i dx_ij sum_b conj(a_ib) x_jb,
// gH[i*ldH + slot] += (Re g, -Im g)
hipError_t launch_velocity_entry_grad(const DevMat& A, int hop_mode, int B, const double2* a, const double2* x,
                                      double* gH, int ldH, hipStream_t s);
// Hermitian tie of per-entry gradients [n][ldH] (re, im): an entry (i, s) -> j and the
// q-th entry of row j pointing back to i (q = its occurrence among row i's entries to j)
// give out = (re_is + re_jp, im_is - im_jp); entries without a partner are copied
hipError_t launch_tie_entries(const DevMat& A, int hop_mode, int64_t n, int ldH, const double* in, double* out,
                              hipStream_t s);
hipError_t launch_adjoint_step(const DevMat& A, int hop_mode, int B, int nc, const AdjIO& io,
                               hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
// out[c] += sum_g gcp[g*nc + c] for c < n_out (fixed order)
hipError_t launch_reduce_classes(const double* gcp, int G, int nc, int n_out, double* out,
                                 hipStream_t s);

// out = a deterministic unit-modulus vector (timing input of gpuqt_autotune).
hipError_t launch_fill_phase(const DevMat& A, int B, double2* out, hipStream_t s);

// Table J[s*ldJ + m] =(2 - delta_m0) J_m(DeltaE_s |dt|), m < Np, s < n_seg.
hipError_t launch_bessel_table(const double* seg_dE, int n_seg, double abs_dt, int Np, int ldJ,
                               double* J, hipStream_t s);

// Final deterministic reduction of per-workgroup partials:
//   partials laid out [M][G][B]; result for (seg, b, k) = sum over the
//   workgroups of seg in increasing order (tree inside one workgroup).
//   mode 0: complex out[(seg*B + b)*M + k];
//   mode 1: real part into out_real[(seg*B + b)*M + k].
//   sym: the rows hold raw dots of launch_moment_step_sym; moment k >= 2 is
//   2 row_k - moment_{k mod 2}.
hipError_t launch_reduce_moments(const double2* part, int M, int G, int B, int n_seg,
                                 const int32_t* seg_blk0_dev, int sym, double2* out, double* out_real,
                                 hipStream_t s);

// Moment step of a Hermitian set (phiL = phiR = v_0) by the product identities
// T_{2k} = 2 T_k^2 - T_0 and T_{2k-1} = 2 T_k T_{k-1} - T_1: writes the raw
// per-workgroup dots <v_k|v_{k-1}> to part_a and <v_k|v_k> to part_c; the first
// step writes <v_0|v_0> to part_a, <v_0|v_1> to part_b and <v_1|v_1> to part_c.
hipError_t launch_moment_step_sym(const DevMat& A, int hop_mode, int B, const StepIO& io,
                                  double2* part_a, double2* part_b, double2* part_c, hipStream_t s);

// The same for <a|T_n|b>, a != b: chains a (xa, wa -> oa) and b (xb, wb -> ob)
// advance together; raw dots <a_k|b_{k-1}> -> part_a, <a_k|b_k> -> part_c, and on
// the first step <a|b> -> part_a, <a|b_1> -> part_b, <a_1|b_1> -> part_c.
struct ChainIO;
hipError_t launch_moment_step_pair(const DevMat& A, int hop_mode, int B, const ChainIO& io,
                                   double2* part_a, double2* part_b, double2* part_c, hipStream_t s);

// out[r][e] = pref_base / sqrt(1 - x^2) * sum_n g_n (2 - delta_n0) T_n(x) C[r][n],
// x = E[e] * inv_dE (NaN where |x| >= 1).
hipError_t launch_kpm(int R, int M, const double* C, int n_E, const double* E, double inv_dE,
                      double pref_base, int jackson, double* out, hipStream_t s);

// out[r][n] = sum_e g[r][e] d(KPM sum)[r][e] / dC[r][n]   (transpose of launch_kpm)
hipError_t launch_kpm_adjoint(int R, int M, const double* g, int n_E, const double* E, double inv_dE,
                              double pref_base, int jackson, double* out, hipStream_t s);

hipError_t launch_copy(const double2* src, double2* dst, size_t n16, hipStream_t s);

}  // namespace gpuqt
