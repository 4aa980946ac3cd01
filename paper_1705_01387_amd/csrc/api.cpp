// C ABI of the transport library: handles, workspace layout, argument checks,
// and the host-side sequencing of the Chebyshev recurrences (Sections 3.2-3.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "bessel.h"
#include "internal.h"

using namespace gpuqt;

namespace gpuqt {
// Reverse step of a Hermitian moment set (kernels_adjoint.hip): the two-chain
// step with both chains equal, one chain gathered; the b fields of io unused.
hipError_t launch_adjoint_sym_step(const DevMat& A, int hop_mode, int B, int nc, const AdjPairIO& io,
                                   hipStream_t s);
}  // namespace gpuqt

namespace {

thread_local std::string g_err;

gpuqt_status fail(gpuqt_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

}  // namespace

gpuqt_status gpuqt::set_error(gpuqt_status st, const std::string& msg) { return fail(st, msg); }

namespace {

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(GPUQT_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kAutoNpCap = 8192;
// autotuner: Chebyshev steps per timing, and the workspace that also lets it
// time the two-chain moment, two-vector evolution and MSD families
constexpr int kTuneSteps = 24;
constexpr int kTuneNp = 13;
constexpr int kTuneVectors = 8;

bool valid_B(int B) { return B == 1 || B == 2 || B == 4 || B == 8 || B == 16; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace layout: nv vectors [n][B] c128, then np rows of per-workgroup
// partials [G][B] c128, then the Bessel table [n_seg][ldJ] double.
struct WsLayout {
  size_t vec_bytes = 0;
  size_t off_part = 0;
  size_t off_J = 0;
  size_t total = 0;
};

WsLayout ws_layout(const Handle* h, int nv, int B, int64_t part_rows, int64_t ldJ) {
  WsLayout L;
  L.vec_bytes = round_up((size_t)h->n * (size_t)B * 16u, 256);
  L.off_part = L.vec_bytes * (size_t)nv;
  const size_t part = round_up((size_t)part_rows * (size_t)h->G * (size_t)B * 16u, 256);
  L.off_J = L.off_part + part;
  L.total = L.off_J + round_up((size_t)h->n_seg * (size_t)ldJ * 8u, 256);
  return L;
}

int op_vectors(int op) {
  switch (op) {
    case GPUQT_OP_MOMENTS: return 4;
    case GPUQT_OP_EVOLVE: return 2;
    case GPUQT_OP_EVOLVE_COMMUTATOR: return 5;
    case GPUQT_OP_VAC: return 9;
    case GPUQT_OP_MSD: return 9;
    case GPUQT_OP_MOMENTS_BACKWARD: return 6;
    case GPUQT_OP_AUTOTUNE: return kTuneVectors;
    default: return -1;
  }
}

gpuqt_status check_device(const Handle* h) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != h->device)
    return fail(GPUQT_ERR_HIP, "handle was built on device " + std::to_string(h->device) +
                                   " but device " + std::to_string(dev) + " is current");
  return GPUQT_OK;
}

gpuqt_status check_vec(const double* p, const char* name) {
  if (!p) return fail(GPUQT_ERR_ARG, std::string(name) + " is NULL");
  if (!aligned16(p)) return fail(GPUQT_ERR_ARG, std::string(name) + " is not 16-byte aligned");
  return GPUQT_OK;
}

bool overlap(const void* a, const void* b, size_t bytes) {
  if (!a || !b) return false;
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

int auto_terms_host(double tau) {
  if (!(tau >= 0) || !std::isfinite(tau)) return -1;
  int m0 = (int)std::floor(tau) + 1;
  int cap = m0 + 64 + (int)(16.0 * std::cbrt(tau + 1.0));
  for (;;) {
    std::vector<double> J(cap);
    bessel_miller(tau, cap, J.data());
    for (int m = m0; m < cap; ++m)
      if (std::fabs(J[m]) < 1e-16) return m;
    cap *= 2;
    if (cap > (1 << 26)) return -1;
  }
}

int terms_for(const Handle* h, double dt, int Np) {
  if (Np > 0) return Np;
  int best = 1;
  for (double e : h->seg_dE) best = std::max(best, auto_terms_host(e * std::fabs(dt)));
  return best;
}

// checkpoint stride of the moments adjoint: 1 keeps every forward vector (no
// recomputation), >= 2 as given, 0 chooses ceil(sqrt(M))
int backward_stride(int M, int stride) {
  if (stride >= 1) return stride;
  int s = (int)std::ceil(std::sqrt((double)std::max(M, 1)));
  return std::max(2, s);
}

// checkpoint pairs of the backward pass (none when every vector is kept)
int backward_pairs(int M, int s) { return (M >= 2 && s >= 2) ? (M - 1 + s - 1) / s : 0; }

// steps of the two-chain (product identity) form of an M-moment set
int pair_steps(int M) { return std::max(1, M / 2); }

// vectors of the backward workspace: 3 forward, 3 adjoint, 2 per checkpoint
// pair and s recomputed (s >= 2); with every vector kept (s = 1) the two-chain
// reverse: both chains' K forward vectors and 3 adjoint vectors per chain
int backward_vectors(int M, int s) {
  if (s == 1) return 6 + 2 * pair_steps(M);
  return 6 + 2 * backward_pairs(M, s) + s;
}

// doubles per segment of the raw-dot weights of the two-chain reverse
int64_t raw_weight_len(int B, int M) { return (int64_t)B * (2 * pair_steps(M) + 2); }

int class_stride(int n_class) { return n_class <= 1 ? 1 : (n_class <= 2 ? 2 : 4); }

// ---------------------------------------------------------------------------
// sequencing helpers (enqueue only; arguments already checked)
// ---------------------------------------------------------------------------

// partial rows a moment call needs (the symmetric form writes up to row M)
int moment_rows(int M) { return std::max(M + 1, 3); }

// Opt-in timing: events around a run of `launches` launches of one family.
struct TimeScope {
  const Handle* h;
  hipStream_t s;
  Handle::TimingRec rec{};
  bool on = false;
  TimeScope(const Handle* hh, hipStream_t ss, int family, int64_t launches) : h(hh), s(ss) {
    if (!h->timing || launches <= 0) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    rec.family = family;
    rec.launches = launches;
    if (hipEventCreate(&rec.a) != hipSuccess) return;
    if (hipEventCreate(&rec.b) != hipSuccess) {
      (void)hipEventDestroy(rec.a);
      return;
    }
    on = hipEventRecord(rec.a, s) == hipSuccess;
  }
  ~TimeScope() {
    if (!on) return;
    if (hipEventRecord(rec.b, s) == hipSuccess) {
      h->timing_recs.push_back(rec);
    } else {
      (void)hipEventDestroy(rec.a);
      (void)hipEventDestroy(rec.b);
    }
  }
};

// M moments into part rows 0..M-1 using buffers A, Bf.  sym (phiL = phiR):
// ceil((M-1)/2) steps of k_moment_step_sym leave raw dots that the reduction
// in symmetric mode turns into the moments.
gpuqt_status run_moments(const Handle* h, int B, const double2* phiL, const double2* phiR, int M,
                         double2* part, double2* A, double2* Bf, hipStream_t s, bool sym = false,
                         double2* A2 = nullptr, double2* B2 = nullptr, double2* const* keep = nullptr) {
  const int fam = A2 || keep ? FAM_PAIR : sym ? FAM_SYM : FAM_MOMENT;
  const DevMat D = h->view(B, fam);
  const int64_t row = (int64_t)D.G * B;   // partial rows: one per logical workgroup of this plan
  if (A2 || keep) {   // pair: chains phiL (A, Bf) and phiR (A2, B2), product identities
    const int K = std::max(1, M / 2);
    // keep: every chain vector goes to its own buffer, a_k to keep[k-1], b_k to keep[K+k-1]
    if (keep) {
      A = keep[0];
      A2 = keep[K];
    }
    TimeScope ts(h, s, 2, K);
    ChainIO io{phiL, nullptr, A, phiR, nullptr, A2, 1, 1};
    HIP_TRY(launch_moment_step_pair(D, h->hop_mode, B, io, part, part + row, part + 2 * row, s));
    const double2 *pa = phiL, *pb = phiR;
    double2 *ca = A, *cb = A2;
    for (int k = 2; k <= K; ++k) {
      double2* oa = keep ? keep[k - 1] : (pa == phiL) ? Bf : const_cast<double2*>(pa);
      double2* ob = keep ? keep[K + k - 1] : (pb == phiR) ? B2 : const_cast<double2*>(pb);
      ChainIO st{ca, pa, oa, cb, pb, ob, 0, 1};
      HIP_TRY(launch_moment_step_pair(D, h->hop_mode, B, st, part + row * (2 * k - 1), nullptr,
                                      part + row * (2 * k), s));
      pa = ca;
      pb = cb;
      ca = oa;
      cb = ob;
    }
    return GPUQT_OK;
  }
  if (sym) {
    const int K = std::max(1, M / 2);   // ceil((M-1)/2), at least the first step
    TimeScope ts(h, s, 1, K);
    StepIO io{phiR, nullptr, A, 1};
    HIP_TRY(launch_moment_step_sym(D, h->hop_mode, B, io, part, part + row, part + 2 * row, s));
    const double2* prev = phiR;
    double2* cur = A;
    for (int k = 2; k <= K; ++k) {
      double2* out = (prev == phiR) ? Bf : const_cast<double2*>(prev);
      StepIO st{cur, prev, out, 0};
      HIP_TRY(launch_moment_step_sym(D, h->hop_mode, B, st, part + row * (2 * k - 1), nullptr,
                                     part + row * (2 * k), s));
      prev = cur;
      cur = out;
    }
    return GPUQT_OK;
  }
  TimeScope ts(h, s, 0, std::max(1, M - 1));
  StepIO io{phiR, nullptr, A, 1};
  HIP_TRY(launch_moment_step(D, h->hop_mode, B, io, phiL, part + row, part, s));
  const double2* prev = phiR;
  double2* cur = A;
  for (int k = 2; k < M; ++k) {
    double2* out = (prev == phiR) ? Bf : const_cast<double2*>(prev);
    StepIO st{cur, prev, out, 0};
    HIP_TRY(launch_moment_step(D, h->hop_mode, B, st, phiL, part + row * k, nullptr, s));
    prev = cur;
    cur = out;
  }
  return GPUQT_OK;
}

double2 phase_pow(int m, double sgn) {
  // (-i sgn)^m
  switch (m & 3) {
    case 0: return make_double2(1.0, 0.0);
    case 1: return make_double2(0.0, -sgn);
    case 2: return make_double2(-1.0, 0.0);
    default: return make_double2(0.0, sgn);
  }
}

// psi_out = U(dt) psi_in; when chi_out: chi_out = [X,U(dt)] psi_in + U(dt) chi_in.
// Buffers: aA, aB always; bA, bB, zero when chi_out.  Jtab: [n_seg][Np].
gpuqt_status run_evolve(const Handle* h, int B, double dt, int Np, const double2* psi_in,
                        double2* psi_out, const double2* chi_in, double2* chi_out, double2* aA,
                        double2* aB, double2* bA, double2* bB, double2* zero, double* Jtab,
                        hipStream_t s) {
  const DevMat D = h->view(B);
  const double sgn = dt >= 0 ? 1.0 : -1.0;
  HIP_TRY(launch_bessel_table(h->d_seg_dE, h->n_seg, std::fabs(dt), Np, Np, Jtab, s));
  const double2 ph0 = phase_pow(0, sgn);
  if (!chi_out) {
    if (Np == 1) {
      HIP_TRY(launch_scale(D, B, psi_in, psi_out, Jtab, Np, s));
      return GPUQT_OK;
    }
    TimeScope ts(h, s, 3, Np - 1);
    const DevMat E = h->view(B, FAM_EVOLVE);
    StepIO io{psi_in, nullptr, aA, 1};
    HIP_TRY(launch_evolve_term(E, h->hop_mode, B, io, psi_out, Jtab, Np, 1, phase_pow(1, sgn), ph0, s));
    const double2* prev = psi_in;
    double2* cur = aA;
    for (int m = 2; m < Np; ++m) {
      double2* out = (prev == psi_in) ? aB : const_cast<double2*>(prev);
      StepIO st{cur, prev, out, 0};
      HIP_TRY(launch_evolve_term(E, h->hop_mode, B, st, psi_out, Jtab, Np, m, phase_pow(m, sgn), ph0, s));
      prev = cur;
      cur = out;
    }
    return GPUQT_OK;
  }
  const double2* b0 = chi_in;
  if (!b0) {
    HIP_TRY(launch_scale(D, B, nullptr, zero, Jtab, Np, s));  // zero fill
    b0 = zero;
  }
  if (Np == 1) {
    HIP_TRY(launch_scale(D, B, psi_in, psi_out, Jtab, Np, s));
    HIP_TRY(launch_scale(D, B, b0, chi_out, Jtab, Np, s));
    return GPUQT_OK;
  }
  TimeScope ts(h, s, 4, Np - 1);
  const DevMat E = h->view(B, FAM_MSD);
  ChainIO io{psi_in, nullptr, aA, b0, nullptr, bA, 1, 1};
  HIP_TRY(launch_msd_term(E, h->hop_mode, B, io, psi_out, chi_out, Jtab, Np, 1, phase_pow(1, sgn), ph0, s));
  const double2 *pa = psi_in, *pb = b0;
  double2 *ca = aA, *cb = bA;
  for (int m = 2; m < Np; ++m) {
    double2* oa = (pa == psi_in) ? aB : const_cast<double2*>(pa);
    double2* ob = (pb == chi_in || pb == zero) ? bB : const_cast<double2*>(pb);
    ChainIO st{ca, pa, oa, cb, pb, ob, 0, 1};
    HIP_TRY(launch_msd_term(E, h->hop_mode, B, st, psi_out, chi_out, Jtab, Np, m, phase_pow(m, sgn), ph0, s));
    pa = ca;
    pb = cb;
    ca = oa;
    cb = ob;
  }
  return GPUQT_OK;
}

// a_out = U(dt) a_in and b_out = U(dt) b_in with one matrix read per term
// (scratch aA, aB, bA, bB; outputs must not alias the inputs).
gpuqt_status run_evolve_pair(const Handle* h, int B, double dt, int Np, const double2* a_in, double2* a_out,
                             const double2* b_in, double2* b_out, double2* aA, double2* aB, double2* bA,
                             double2* bB, double* Jtab, hipStream_t s, double2* const* keep = nullptr) {
  // keep: every chain vector to its own buffer, a_m to keep[m-1], b_m to keep[Np-1+m-1]
  const double sgn = dt >= 0 ? 1.0 : -1.0;
  HIP_TRY(launch_bessel_table(h->d_seg_dE, h->n_seg, std::fabs(dt), Np, Np, Jtab, s));
  if (Np == 1) {
    const DevMat D = h->view(B);
    HIP_TRY(launch_scale(D, B, a_in, a_out, Jtab, Np, s));
    HIP_TRY(launch_scale(D, B, b_in, b_out, Jtab, Np, s));
    return GPUQT_OK;
  }
  const double2 ph0 = phase_pow(0, sgn);
  TimeScope ts(h, s, FAM_EVOLVE_PAIR, Np - 1);
  const DevMat E = h->view(B, FAM_EVOLVE_PAIR);
  if (keep) {
    aA = keep[0];
    bA = keep[Np - 1];
  }
  ChainIO io{a_in, nullptr, aA, b_in, nullptr, bA, 1, 1};
  HIP_TRY(launch_evolve_pair_term(E, h->hop_mode, B, io, a_out, b_out, Jtab, Np, 1, phase_pow(1, sgn), ph0, s));
  const double2 *pa = a_in, *pb = b_in;
  double2 *ca = aA, *cb = bA;
  for (int m = 2; m < Np; ++m) {
    double2* oa = keep ? keep[m - 1] : (pa == a_in) ? aB : const_cast<double2*>(pa);
    double2* ob = keep ? keep[Np - 1 + m - 1] : (pb == b_in) ? bB : const_cast<double2*>(pb);
    ChainIO st{ca, pa, oa, cb, pb, ob, 0, 1};
    HIP_TRY(launch_evolve_pair_term(E, h->hop_mode, B, st, a_out, b_out, Jtab, Np, m, phase_pow(m, sgn), ph0, s));
    pa = ca;
    pb = cb;
    ca = oa;
    cb = ob;
  }
  return GPUQT_OK;
}

// Source of the adjoint recurrence: real loss weights w[seg][b][n] on Re mu_n,
// or the complex coefficients c_n = J[seg][n] (-i sgn)^n of an evolution series
// (the adjoint source is conj(c_n) phiL).
struct BwdSource {
  const double* wts = nullptr;
  const double* Jtab = nullptr;
  int ldJ = 0;
  double sgn = 1.0;
};

// Reverse of the M-step recurrence started at phiR, with phiL the adjoint
// source: when gU is set, parameter terms go to gU, (nc > 0) gcp and (gH set)
// the per-entry gradients [n][max_nn] (re, im), with the
// forward vectors recomputed from checkpoints every s steps; lam0 (if set)
// receives sum_n conj(c_n) T_n phiL (accumulated when acc0).  vec: at least
// backward_vectors(M, s) workspace vectors.
gpuqt_status run_backward(const Handle* h, int B, const double2* pL, const double2* pR, int M,
                          const BwdSource& src, double* gU, double* gcp, int nc, double2* lam0,
                          bool acc0, int s, double2* const* vec, hipStream_t sm,
                          double2* const* recorded = nullptr, double* gH = nullptr) {
  // recorded (s = 1 with parameter terms): v_1 .. v_{M-2} = T_n pR already computed
  const DevMat D = h->view(B);                  // adjoint steps: primary plan (class partials)
  const DevMat F = h->view(B, FAM_MOMENT);      // forward recomputation: no partials
  const bool grad = gU != nullptr;
  const int K = backward_pairs(M, s);
  double2* const* R = vec;
  double2* const* Lm = vec + 3;
  auto ck = [&](int k, int q) { return vec[6 + 2 * k + q]; };
  auto sb = [&](int j) { return vec[6 + 2 * K + j]; };
  auto make = [&](int n) {
    AdjIO a;
    a.x = (n + 1 <= M - 1) ? Lm[(n + 1) % 3] : nullptr;
    a.w = (n + 2 <= M - 1) ? Lm[(n + 2) % 3] : nullptr;
    a.out = Lm[n % 3];
    a.phiL = pL;
    a.wts = src.wts;
    a.M = M;
    a.n = n;
    a.f_rec = 2.0;
    a.v = nullptr;
    a.f = n == 1 ? 1.0 : 2.0;
    a.gU = gU;
    a.gcp = gcp;
    a.cls = h->d_cls;
    a.gH = gU ? gH : nullptr;
    a.ldH = h->max_nn_in;
    a.Jtab = src.Jtab;
    a.ldJ = src.ldJ;
    a.accumulate = 0;
    const double2 p = phase_pow(n, src.sgn);
    a.src_phase = make_double2(p.x, -p.y);   // conj((-i sgn)^n)
    return a;
  };
  if (grad && s == 1) {
    // forward: v_1 .. v_{M-2}, every one kept (v_n in sb(n), unless recorded);
    // then the reverse
    auto fwd = [&](int n) -> const double2* { return n == 0 ? pR : recorded ? recorded[n - 1] : sb(n); };
    if (!recorded) {
      const double2* prev2 = nullptr;
      const double2* prev1 = pR;
      for (int n = 1; n <= M - 2; ++n) {
        StepIO io{prev1, prev2, sb(n), n == 1 ? 1 : 0};
        HIP_TRY(launch_moment_step(F, h->hop_mode, B, io, nullptr, nullptr, nullptr, sm));
        prev2 = prev1;
        prev1 = sb(n);
      }
    }
    for (int n = M - 1; n >= 1; --n) {
      AdjIO a = make(n);
      a.v = fwd(n - 1);
      HIP_TRY(launch_adjoint_step(D, h->hop_mode, B, nc, a, sm));
    }
  } else if (grad) {
    // forward: v_1 .. v_{M-2}, keeping v_{ks} and v_{ks+1} as checkpoints
    const double2* prev2 = nullptr;
    const double2* prev1 = pR;
    for (int n = 1; n <= M - 2; ++n) {
      double2* out = (n % s == 0 || n % s == 1) ? ck(n / s, n % s) : R[n % 3];
      StepIO io{prev1, prev2, out, n == 1 ? 1 : 0};
      HIP_TRY(launch_moment_step(F, h->hop_mode, B, io, nullptr, nullptr, nullptr, sm));
      prev2 = prev1;
      prev1 = out;
    }
    auto slot = [&](int k, int j) -> const double2* {
      if (j == 0) return k == 0 ? pR : ck(k, 0);
      if (j == 1) return ck(k, 1);
      return sb(j);
    };
    for (int k = K - 1; k >= 0; --k) {
      const int lo = k * s + 1, hi = std::min((k + 1) * s, M - 1);
      for (int j = 2; j <= hi - 1 - k * s; ++j) {   // recompute v_{ks+j}
        StepIO io{slot(k, j - 1), slot(k, j - 2), sb(j), 0};
        HIP_TRY(launch_moment_step(F, h->hop_mode, B, io, nullptr, nullptr, nullptr, sm));
      }
      for (int n = hi; n >= lo; --n) {
        AdjIO a = make(n);
        a.v = slot(k, n - 1 - k * s);
        HIP_TRY(launch_adjoint_step(D, h->hop_mode, B, nc, a, sm));
      }
    }
  } else {
    for (int n = M - 1; n >= 1; --n) {
      AdjIO a = make(n);
      HIP_TRY(launch_adjoint_step(D, h->hop_mode, B, 0, a, sm));
    }
  }
  if (lam0) {   // lam_0 = conj(c_0) phiL + H~ lam_1 - lam_2 = sum_n conj(c_n) T_n(H~) phiL
    AdjIO a = make(0);
    a.x = M >= 2 ? Lm[1] : nullptr;
    a.w = M >= 3 ? Lm[2] : nullptr;
    a.out = lam0;
    a.f_rec = 1.0;
    a.gU = nullptr;
    a.gcp = nullptr;
    a.gH = nullptr;
    a.accumulate = acc0 ? 1 : 0;
    HIP_TRY(launch_adjoint_step(D, h->hop_mode, B, 0, a, sm));
  }
  return GPUQT_OK;
}


// Reverse of the two-chain moment computation with every forward vector kept:
// chains a_k = T_k pL and b_k = T_k pR over K = pair_steps(M) steps, loss
// weights wts [seg][B][M] on Re mu_n turned into raw-dot weights om.  When gU
// is set, parameter terms go to gU and (nc > 0) gcp.  abar_0 = sum_n w_n T_n pR
// (the adjoint of pL) goes to outA and bbar_0 = sum_n w_n T_n pL (the adjoint of
// pR) to outB when they are set, added to them when accA / accB.
// vec: backward_vectors(M, 1) vectors; om: n_seg * raw_weight_len(B, M) doubles;
// scratch: 3 partial rows (G x B each) that the forward two-chain steps fill and
// nobody reads.
gpuqt_status run_backward_pair(const Handle* h, int B, const double2* pL, const double2* pR, int M,
                               const double* wts, double* gU, double* gcp, int nc, double2* outA,
                               bool accA, double2* outB, bool accB, double2* const* vec, double* om,
                               double2* scratch, hipStream_t sm, double2* const* recorded = nullptr) {
  const int K = pair_steps(M);
  const int R = 2 * K + 2;
  HIP_TRY(launch_raw_weights(wts, h->n_seg * B, M, R, om, sm));
  // forward chains a_1..a_K, b_1..b_K: recorded by the forward call, or computed here into vec
  double2* const* ch = recorded ? recorded : vec;
  auto fa = [&](int k) -> const double2* { return k == 0 ? pL : ch[k - 1]; };
  auto fb = [&](int k) -> const double2* { return k == 0 ? pR : ch[K + k - 1]; };
  if (!recorded) {
    TimeScope ts(h, sm, FAM_PAIR, K);
    const DevMat F = h->view(B, FAM_PAIR);
    const int64_t row = (int64_t)F.G * B;
    for (int k = 1; k <= K; ++k) {
      ChainIO io{fa(k - 1), k >= 2 ? fa(k - 2) : nullptr, vec[k - 1],
                 fb(k - 1), k >= 2 ? fb(k - 2) : nullptr, vec[K + k - 1], k == 1 ? 1 : 0, 1};
      HIP_TRY(launch_moment_step_pair(F, h->hop_mode, B, io, scratch, scratch + row, scratch + 2 * row, sm));
    }
  }
  double2* const* La = recorded ? vec : vec + 2 * K;   // rotating abar
  double2* const* Lb = La + 3;                         // rotating bbar
  const DevMat D = h->view(B);            // class partials over the primary plan
  for (int k = K; k >= 0; --k) {
    if (k == 0 && !outA && !outB) break;
    AdjPairIO io{};
    io.xa = k + 1 <= K ? La[(k + 1) % 3] : nullptr;
    io.wa = k + 2 <= K ? La[(k + 2) % 3] : nullptr;
    io.xb = k + 1 <= K ? Lb[(k + 1) % 3] : nullptr;
    io.wb = k + 2 <= K ? Lb[(k + 2) % 3] : nullptr;
    io.oa = (k == 0 && outA) ? outA : La[k % 3];
    io.ob = (k == 0 && outB) ? outB : Lb[k % 3];
    io.acc_a = (k == 0 && outA && accA) ? 1 : 0;
    io.acc_b = (k == 0 && outB && accB) ? 1 : 0;
    io.a_m1 = k >= 1 ? fa(k - 1) : nullptr;
    io.a_k = fa(k);
    io.a_p1 = k + 1 <= K ? fa(k + 1) : nullptr;
    io.b_m1 = k >= 1 ? fb(k - 1) : nullptr;
    io.b_k = fb(k);
    io.om = om;
    io.R = R;
    io.k = k;
    io.f_rec = k >= 1 ? 2.0 : 1.0;
    io.f = k >= 2 ? 2.0 : 1.0;
    io.gU = gU;
    io.gcp = gcp;
    io.cls = h->d_cls;
    HIP_TRY(launch_adjoint_pair_step(D, h->hop_mode, B, gU ? nc : 0, io, sm));
  }
  return GPUQT_OK;
}

// Reverse of a Hermitian moment set (phiL = phiR = phi) in the product-identity
// form: the chain a_k = T_k phi (k = 1..K) into vec[0..K-1], then the reverse
// of cbar_k = abar_k + bbar_k in three rotating vectors vec[K..K+2]; lam0 (if
// set) receives sum_n w_n T_n phi.  Half the vectors and half the gathers of
// run_backward_pair with both arguments equal.
gpuqt_status run_backward_sym(const Handle* h, int B, const double2* ph, int M, const double* wts, double* gU,
                              double* gcp, int nc, double2* lam0, bool acc0, double2* const* vec, double* om,
                              double2* scratch, hipStream_t sm) {
  const int K = pair_steps(M);
  const int R = 2 * K + 2;
  HIP_TRY(launch_raw_weights(wts, h->n_seg * B, M, R, om, sm));
  auto fa = [&](int k) -> const double2* { return k == 0 ? ph : vec[k - 1]; };
  {
    TimeScope ts(h, sm, FAM_SYM, K);
    const DevMat F = h->view(B, FAM_SYM);
    const int64_t row = (int64_t)F.G * B;
    for (int k = 1; k <= K; ++k) {
      StepIO io{fa(k - 1), k >= 2 ? fa(k - 2) : nullptr, vec[k - 1], k == 1 ? 1 : 0};
      HIP_TRY(launch_moment_step_sym(F, h->hop_mode, B, io, scratch, scratch + row, scratch + 2 * row, sm));
    }
  }
  double2* const* Lc = vec + K;   // rotating cbar
  const DevMat D = h->view(B);     // class partials over the primary plan
  for (int k = K; k >= 0; --k) {
    if (k == 0 && !lam0) break;
    AdjPairIO io{};
    io.xa = k + 1 <= K ? Lc[(k + 1) % 3] : nullptr;
    io.wa = k + 2 <= K ? Lc[(k + 2) % 3] : nullptr;
    io.oa = (k == 0) ? lam0 : Lc[k % 3];
    io.acc_a = (k == 0 && acc0) ? 1 : 0;
    io.a_m1 = k >= 1 ? fa(k - 1) : nullptr;
    io.a_k = fa(k);
    io.a_p1 = k + 1 <= K ? fa(k + 1) : nullptr;
    io.om = om;
    io.R = R;
    io.k = k;
    io.f_rec = k >= 1 ? 2.0 : 1.0;
    io.f = k >= 2 ? 2.0 : 1.0;
    io.gU = gU;
    io.gcp = gcp;
    io.cls = h->d_cls;
    HIP_TRY(launch_adjoint_sym_step(D, h->hop_mode, B, gU ? nc : 0, io, sm));
  }
  return GPUQT_OK;
}

}  // namespace

extern "C" {

const char* gpuqt_last_error(void) { return g_err.c_str(); }

gpuqt_status gpuqt_jackson(int32_t M, double* g) {
  if (M < 0 || (M > 0 && !g)) return fail(GPUQT_ERR_ARG, "bad arguments to gpuqt_jackson");
  const double a = 1.0 / (M + 1);
  const double cot = std::cos(M_PI * a) / std::sin(M_PI * a);
  for (int n = 0; n < M; ++n)
    g[n] = (1.0 - n * a) * std::cos(M_PI * n * a) + a * std::sin(M_PI * n * a) * cot;
  return GPUQT_OK;
}

gpuqt_status gpuqt_bessel(double tau, int32_t Np, double* J) {
  if (!(tau >= 0) || !std::isfinite(tau) || Np < 0 || (Np > 0 && !J))
    return fail(GPUQT_ERR_ARG, "bad arguments to gpuqt_bessel");
  bessel_miller(tau, Np, J);
  return GPUQT_OK;
}

int32_t gpuqt_auto_terms(double tau) { return auto_terms_host(tau); }

gpuqt_status gpuqt_build_h(const gpuqt_h_desc* desc, void* stream, gpuqt_h* out) {
  if (!out) return fail(GPUQT_ERR_ARG, "out is NULL");
  *out = nullptr;
  HostLayout L;
  std::string msg;
  gpuqt_status st = build_host_layout(desc, &L, &msg);
  if (st != GPUQT_OK) return fail(st, msg);
  int dev = -1, ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) return fail(GPUQT_ERR_HIP, "no HIP device available");
  HIP_TRY(hipGetDevice(&dev));
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));

  Handle* h = new Handle();
  h->device = dev;
  h->n = L.n;
  h->n_seg = L.n_seg;
  h->n_class = L.n_class;
  h->hop_mode = L.hop_mode;
  h->S = L.S;
  h->S_log2 = L.S_log2;
  h->n_slices = L.n_slices;
  h->entries = (int64_t)L.col.size();
  h->nnz = L.nnz;
  h->max_width = L.max_width;
  h->uniform_width = L.uniform_width;
  h->seg_off = L.seg_off;
  h->seg_dE = L.seg_dE;
  h->seg_gersh = L.seg_gersh;
  std::vector<int32_t> seg_blk0;
  plan_blocks(L.seg_off, cus, kPerCU, &h->plan_host, &seg_blk0);
  h->G = (int32_t)h->plan_host.size();

  hipStream_t s = static_cast<hipStream_t>(stream);
  bool ok = true;
  auto up = [&](void** dst, const void* src, size_t bytes) {
    if (!ok || bytes == 0) return;
    if (hipMalloc(dst, bytes) != hipSuccess) {
      ok = false;
      *dst = nullptr;
      return;
    }
    h->device_bytes += bytes;
    if (hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) ok = false;
  };
  up((void**)&h->d_slice_ptr, L.slice_ptr.data(), L.slice_ptr.size() * 8);
  if (L.hop_mode != HOP_DICT)   // the value table holds the column offsets
    up((void**)&h->d_col, L.col.data(), L.col.size() * 4);
  up((void**)&h->d_hop, L.hop.data(), L.hop.size() * 8);
  up((void**)&h->d_dx, L.dx.data(), L.dx.size() * 8);
  up((void**)&h->d_hidx, L.hidx.data(), L.hidx.size() * 2);
  up((void**)&h->d_htab, L.htab.data(), L.htab.size() * 8);
  up((void**)&h->d_dxtab, L.dxtab.data(), L.dxtab.size() * 8);
  up((void**)&h->d_offtab, L.offtab.data(), L.offtab.size() * 4);
  h->dict_size = (int32_t)L.dxtab.size();
  up((void**)&h->d_diag, L.diag.data(), L.diag.size() * 8);
  up((void**)&h->d_cls, L.cls.data(), L.cls.size() * 4);
  up((void**)&h->d_plan, h->plan_host.data(), h->plan_host.size() * sizeof(BlkPlan));
  up((void**)&h->d_seg_blk0, seg_blk0.data(), seg_blk0.size() * 4);
  up((void**)&h->d_seg_dE, L.seg_dE.data(), L.seg_dE.size() * 8);
  up((void**)&h->d_seg_hop, L.seg_hop.data(), L.seg_hop.size() * 8);
  up((void**)&h->d_seg_hop0, L.seg_hop.data(), L.seg_hop.size() * 8);
  h->max_nn_in = desc->max_nn;
  if (L.hop_mode == HOP_UNIFORM && L.n_seg == 1 && L.uniform_width == 6 && detect_box(desc, h->box))
    h->box_msd_ok = box_dx_uniform(L, h->box, &h->box_dx) ? 1 : 0;
  // plans for fewer resident workgroups per CU, and each hot family's occupancy
  h->d_plans[kPerCU - 1] = h->d_plan;
  h->d_blk0s[kPerCU - 1] = h->d_seg_blk0;
  h->Gs[kPerCU - 1] = h->G;
  std::vector<std::vector<BlkPlan>> plans(kPerCU);   // alive until the stream is synchronised
  std::vector<std::vector<int32_t>> blk0s(kPerCU);
  std::vector<int32_t> sheet_host, sheet_zc, sheet_blk0;   // alive until the stream is synchronised
  std::vector<int64_t> sheet_off;
  for (int p = 1; p < kPerCU; ++p) {
    plan_blocks(L.seg_off, cus, p, &plans[p - 1], &blk0s[p - 1]);
    h->Gs[p - 1] = (int32_t)plans[p - 1].size();
    up((void**)&h->d_plans[p - 1], plans[p - 1].data(), plans[p - 1].size() * sizeof(BlkPlan));
    up((void**)&h->d_blk0s[p - 1], blk0s[p - 1].data(), blk0s[p - 1].size() * 4);
  }
  {
    const DevMat D0 = h->view(1);
    for (int f = 0; f < kFamilies; ++f)
      for (int lb = 0; lb < kNumB; ++lb)
        for (int v = 0; v < 2; ++v)
          h->occ[f][lb][v] = (int8_t)std::min(kPerCU, kernel_occupancy(f, D0, h->hop_mode, 1 << lb, v));
  }
  // segments that are all periodic squares with one uniform hopping: the sheet kernel's
  // (Lx, Ly) and first row per segment, and per plan and block width its own split of the
  // plan's workgroups over the segments (by work, not rows) and rows per work item
  if (L.hop_mode == HOP_UNIFORM && h->box[0] == 0 && detect_sheets(desc, L.seg_off, &sheet_host)) {
    const int ns = L.n_seg;
    sheet_off.assign(L.seg_off.begin(), L.seg_off.end() - 1);
    sheet_zc.assign((size_t)kPerCU * kNumB * ns, 1);
    sheet_blk0.assign((size_t)kPerCU * kNumB * (ns + 1), 0);
    std::vector<int32_t> len(ns), b0, zc;
    std::vector<int64_t> cols(ns);
    for (int sg = 0; sg < ns; ++sg) len[sg] = sheet_host[2 * sg + 1];
    for (int p = 0; p < kPerCU; ++p) {
      for (int lb = 1; lb < kNumB; ++lb) {   // blocks of B >= 2
        const int tx = (kSheetCells * kBlock) >> lb;   // cells per strip (kSheetCells per lane)
        for (int sg = 0; sg < ns; ++sg) cols[sg] = (sheet_host[2 * sg] + tx - 1) / tx;
        sheet_split(cols, len, h->Gs[p], &b0, &zc);
        std::copy(zc.begin(), zc.end(), sheet_zc.begin() + ((size_t)p * kNumB + lb) * ns);
        std::copy(b0.begin(), b0.end(), sheet_blk0.begin() + ((size_t)p * kNumB + lb) * (ns + 1));
      }
    }
    up((void**)&h->d_sheet, sheet_host.data(), sheet_host.size() * 4);
    up((void**)&h->d_sheet_off, sheet_off.data(), sheet_off.size() * 8);
    up((void**)&h->d_sheet_zc, sheet_zc.data(), sheet_zc.size() * 4);
    up((void**)&h->d_sheet_blk0, sheet_blk0.data(), sheet_blk0.size() * 4);
    h->sheet_ok = ok ? 1 : 0;
  }
  std::vector<double> zeros_g(h->G, 0.0);
  up((void**)&h->d_bound, zeros_g.data(), zeros_g.size() * 8);
  // banded unit orders, per block width: the row window between the first and
  // last use of a gathered element is 2 D rows in the plain order and 2 W in
  // the banded one; W keeps it (with everything else the step streams per
  // row) within kBandBudget of an XCD's L2
  h->seg_period.assign(L.n_seg, 0);
  for (int sg = 0; sg < L.n_seg; ++sg) h->seg_period[sg] = row_period(L, sg);
  // bytes streamed per stored entry: column index + hopping, or one 16-bit table index
  const int64_t entry_b = L.hop_mode == HOP_DICT ? 2 : 4 + (L.hop_mode == HOP_COMPLEX ? 16 : L.hop_mode == HOP_REAL ? 8 : 0);
  std::vector<std::vector<int32_t>> unit_lists(kNumB);
  for (int lb = 0; lb < kNumB; ++lb) {
    const int64_t B = int64_t(1) << lb;
    const int64_t row_bytes = entry_b * L.max_width + 8 + 48 * B;
    const int64_t W = desc->band_rows > 0 ? desc->band_rows
                                          : std::max<int64_t>(256, kBandBudget / (2 * row_bytes) / 64 * 64);
    h->band_rows[lb] = (int32_t)W;
    // per segment: W where the period exceeds it; by default, for blocks of two
    // or more vectors, also two bands per period where the period is long
    // (>= 1024 rows) but within W, since the plain order's 2 D window of B-wide
    // rows can still outgrow what stays cached while the whole chip's rows are
    // in flight (the autotuner keeps whichever is faster; at B = 1 the window is
    // small and the two-chain and series kernels lost with it)
    std::vector<int64_t> width(L.n_seg, 0);
    bool any = false;
    for (int sg = 0; sg < L.n_seg; ++sg) {
      const int64_t D = h->seg_period[sg];
      if (D > W) width[sg] = W;
      else if (desc->band_rows == 0 && B >= 2 && D >= 1024) width[sg] = D / 2 / 64 * 64;
      any = any || width[sg] > 0;
    }
    if (any) {
      banded_units(L.seg_off, h->seg_period, width, &unit_lists[lb]);
      up((void**)&h->d_units[lb], unit_lists[lb].data(), unit_lists[lb].size() * 4);
    }
    // pencil order: the reuse window between a row and its neighbours one period
    // on spans kPencil bands of units, so its band width is half the banded one
    const int64_t Wp = desc->band_rows > 0 ? desc->band_rows
                                           : std::max<int64_t>(256, kBandBudget / (4 * row_bytes) / 64 * 64);
    h->pencil_rows[lb] = (int32_t)Wp;
    std::vector<int64_t> pw(L.n_seg, 0);
    bool anyp = false;
    for (int sg = 0; sg < L.n_seg; ++sg) {
      if (h->seg_period[sg] >= 128) pw[sg] = Wp;
      anyp = anyp || pw[sg] > 0;
    }
    if (anyp) {
      std::vector<int32_t> pl;
      pencil_units(L.seg_off, h->seg_period, pw, &pl);
      up((void**)&h->d_units_p[lb], pl.data(), pl.size() * 4);
    }
  }
  h->seg_hop0 = L.seg_hop;
  h->class_scale.assign(h->n_class, 1.0);
  if (ok && hipStreamSynchronize(s) != hipSuccess) ok = false;
  if (!ok) {
    gpuqt_destroy_h(reinterpret_cast<gpuqt_h>(h));
    return fail(GPUQT_ERR_NOMEM, "device allocation or copy failed while building the layout");
  }
  *out = reinterpret_cast<gpuqt_h>(h);
  return GPUQT_OK;
}

void gpuqt_destroy_h(gpuqt_h hh) {
  Handle* h = reinterpret_cast<Handle*>(hh);
  if (!h) return;
  void* ptrs[] = {h->d_slice_ptr, h->d_col, h->d_hop, h->d_dx, h->d_diag, h->d_cls,
                  h->d_plan, h->d_seg_blk0, h->d_seg_dE, h->d_seg_hop, h->d_seg_hop0, h->d_hop0, h->d_bound,
                  h->d_hidx, h->d_htab, h->d_htab0, h->d_dxtab, h->d_offtab, h->d_sheet, h->d_sheet_zc,
                  h->d_sheet_off, h->d_sheet_blk0};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int32_t* p : h->d_units)
    if (p) (void)hipFree(p);
  for (int32_t* p : h->d_units_p)
    if (p) (void)hipFree(p);
  for (int p = 0; p + 1 < kPerCU; ++p) {   // the last entries alias d_plan / d_seg_blk0
    if (h->d_plans[p]) (void)hipFree(h->d_plans[p]);
    if (h->d_blk0s[p]) (void)hipFree(h->d_blk0s[p]);
  }
  for (auto& r : h->timing_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  delete h;
}

gpuqt_status gpuqt_h_info(gpuqt_h hh, gpuqt_h_info_t* info, double* energy_max, double* gershgorin) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h || !info) return fail(GPUQT_ERR_ARG, "NULL handle or info");
  std::memset(info, 0, sizeof(*info));
  info->n = h->n;
  info->n_segments = h->n_seg;
  info->n_class = h->n_class;
  info->hop_mode = h->hop_mode;
  info->slice_height = h->S;
  info->n_slices = h->n_slices;
  info->entries = h->entries;
  info->nnz = h->nnz;
  info->max_width = h->max_width;
  info->uniform_width = h->uniform_width;
  info->grid_blocks = h->G;
  info->device_bytes = h->device_bytes;
  info->kernel_variant = h->variant_code();
  info->family_caps = h->family_caps_code();
  info->max_nn = h->max_nn_in;
  for (int q = 0; q < 3; ++q) info->box[q] = h->box[q];
  info->box_msd = h->box_msd_ok;
  info->sheets = h->sheet_ok;
  info->row_period = 0;
  for (int64_t D : h->seg_period) info->row_period = std::max(info->row_period, D);
  info->banded_mask = 0;
  for (int b = 0; b < kNumB; ++b)
    if (h->d_units[b]) info->banded_mask |= 1 << b;
  info->pencil_mask = 0;
  for (int b = 0; b < kNumB; ++b)
    if (h->d_units_p[b]) info->pencil_mask |= 1 << b;
  for (int s = 0; s < h->n_seg; ++s) {
    if (energy_max) energy_max[s] = h->seg_dE[s];
    if (gershgorin) gershgorin[s] = h->seg_gersh[s];
  }
  return GPUQT_OK;
}

gpuqt_status gpuqt_update_h_values(gpuqt_h hh, const double* onsite, const double* class_scale,
                                   void* stream) {
  Handle* h = reinterpret_cast<Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (onsite && (reinterpret_cast<uintptr_t>(onsite) & 7u))
    return fail(GPUQT_ERR_ARG, "onsite is not 8-byte aligned");
  if (class_scale) {
    if (h->n_class > kMaxUpdateClasses)
      return fail(GPUQT_ERR_UNSUPPORTED, "at most 8 hopping classes can be rescaled");
    for (int c = 0; c < h->n_class; ++c)
      if (!std::isfinite(class_scale[c])) return fail(GPUQT_ERR_ARG, "class_scale is not finite");
  }
  gpuqt_status st;
  if ((st = check_device(h))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const DevMat D = h->view(1);
  if (onsite) HIP_TRY(launch_set_onsite(D, onsite, h->d_diag, s));
  if (class_scale) {
    if (h->hop_mode == HOP_UNIFORM) {
      std::vector<double> v(h->n_seg);
      for (int q = 0; q < h->n_seg; ++q) v[q] = h->seg_hop0[q] * class_scale[0];
      HIP_TRY(hipMemcpyAsync(h->d_seg_hop, v.data(), v.size() * 8, hipMemcpyHostToDevice, s));
      HIP_TRY(hipStreamSynchronize(s));
    } else {
      // per-entry hoppings, or (HOP_DICT) the table of distinct values; classes per
      // entry, or per table entry
      const bool dict = h->hop_mode == HOP_DICT;
      const int64_t count = dict ? h->dict_size : h->entries;
      const bool cplx = dict || h->hop_mode == HOP_COMPLEX;
      double*& cur = dict ? h->d_htab : h->d_hop;
      double*& orig = dict ? h->d_htab0 : h->d_hop0;
      const size_t hb = (size_t)count * (cplx ? 16 : 8);
      if (!orig) {   // first class update: keep the hoppings given at build time
        if (hipMalloc((void**)&orig, hb) != hipSuccess) {
          orig = nullptr;
          return fail(GPUQT_ERR_NOMEM, "could not allocate the copy of the build-time hoppings");
        }
        h->device_bytes += hb;
        HIP_TRY(hipMemcpyAsync(orig, cur, hb, hipMemcpyDeviceToDevice, s));
      }
      ClassScale sc{};
      for (int c = 0; c < h->n_class; ++c) sc.s[c] = class_scale[c];
      HIP_TRY(launch_scale_hops(count, cplx ? 1 : 0, orig, cur, h->n_class > 1 ? h->d_cls : nullptr,
                                sc, s));
    }
    for (int c = 0; c < h->n_class; ++c) h->class_scale[c] = class_scale[c];
  }
  // the spectrum of H / DeltaE must stay in [-1, 1]: recheck the Gershgorin bound
  HIP_TRY(launch_row_bound(D, h->hop_mode, h->d_bound, s));
  std::vector<double> bound(h->G);
  HIP_TRY(hipMemcpyAsync(bound.data(), h->d_bound, bound.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int g = 0; g < h->G; ++g) {
    const int q = h->plan_host[g].seg;
    h->seg_gersh[q] = 0.0;
  }
  for (int g = 0; g < h->G; ++g) {
    const int q = h->plan_host[g].seg;
    h->seg_gersh[q] = std::max(h->seg_gersh[q], bound[g] * h->seg_dE[q]);
  }
  for (int q = 0; q < h->n_seg; ++q)
    if (h->seg_gersh[q] > h->seg_dE[q] * (1.0 + 1e-12))
      return fail(GPUQT_ERR_SPECTRUM, "after the update the Gershgorin bound " +
                                          std::to_string(h->seg_gersh[q]) + " of segment " +
                                          std::to_string(q) + " exceeds its DeltaE " +
                                          std::to_string(h->seg_dE[q]));
  return GPUQT_OK;
}

gpuqt_status gpuqt_workspace_size(gpuqt_h hh, int32_t op, int32_t B, int32_t M, int32_t Np,
                                  size_t* bytes) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h || !bytes) return fail(GPUQT_ERR_ARG, "NULL handle or bytes");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  const int nv = op_vectors(op);
  if (nv < 0) return fail(GPUQT_ERR_ARG, "unknown op");
  if (M < 0 || Np < 0) return fail(GPUQT_ERR_ARG, "M and Np must be >= 0");
  if (op == GPUQT_OP_AUTOTUNE) {
    *bytes = ws_layout(h, kTuneVectors, B, kTuneSteps + 1, kTuneNp).total;
    return GPUQT_OK;
  }
  const bool has_moments = op == GPUQT_OP_MOMENTS || op == GPUQT_OP_VAC || op == GPUQT_OP_MSD ||
                           op == GPUQT_OP_MOMENTS_BACKWARD;
  const bool has_J = op == GPUQT_OP_EVOLVE || op == GPUQT_OP_EVOLVE_COMMUTATOR ||
                     op == GPUQT_OP_VAC || op == GPUQT_OP_MSD;
  const int64_t rows = has_moments ? moment_rows(M) : 0;
  const int64_t ldJ = has_J ? (Np > 0 ? Np : kAutoNpCap) : 0;
  if (op == GPUQT_OP_MOMENTS_BACKWARD) {
    const int s = backward_stride(M, Np);
    *bytes = ws_layout(h, backward_vectors(M, s), B, s == 1 ? 5 : 2, s == 1 ? raw_weight_len(B, M) : 0).total;
    return GPUQT_OK;
  }
  *bytes = ws_layout(h, nv, B, rows, ldJ).total;
  return GPUQT_OK;
}

gpuqt_status gpuqt_moments(gpuqt_h hh, int32_t B, const double* phiL, const double* phiR, int32_t M,
                           double* mu, void* ws, size_t ws_bytes, void* stream) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  if (M < 0) return fail(GPUQT_ERR_ARG, "M must be >= 0");
  if (M == 0) return GPUQT_OK;
  gpuqt_status st;
  if ((st = check_vec(phiL, "phiL")) || (st = check_vec(phiR, "phiR")) || (st = check_vec(mu, "mu")))
    return st;
  const WsLayout W = ws_layout(h, 4, B, moment_rows(M), 0);
  if (!ws || ws_bytes < W.total) return fail(GPUQT_ERR_WORKSPACE, "workspace too small");
  if (!aligned16(ws)) return fail(GPUQT_ERR_ARG, "workspace is not 16-byte aligned");
  if ((st = check_device(h))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  double2* A = reinterpret_cast<double2*>(base);
  double2* Bf = reinterpret_cast<double2*>(base + W.vec_bytes);
  double2* part = reinterpret_cast<double2*>(base + W.off_part);
  const bool sym = phiL == phiR;   // Hermitian set: product identities, half the steps
  if ((st = run_moments(h, B, reinterpret_cast<const double2*>(phiL),
                        reinterpret_cast<const double2*>(phiR), M, part, A, Bf, s, sym,
                        sym ? nullptr : reinterpret_cast<double2*>(base + 2 * W.vec_bytes),
                        sym ? nullptr : reinterpret_cast<double2*>(base + 3 * W.vec_bytes))))
    return st;
  const int fam = sym ? FAM_SYM : FAM_PAIR;
  HIP_TRY(launch_reduce_moments(part, M, h->G_of(B, fam), B, h->n_seg, h->blk0_of(B, fam), 1,   // raw dots
                                reinterpret_cast<double2*>(mu), nullptr, s));
  return GPUQT_OK;
}

gpuqt_status gpuqt_moments_plain(gpuqt_h hh, int32_t B, const double* phiL, const double* phiR, int32_t M,
                                 double* mu, void* ws, size_t ws_bytes, void* stream) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  if (M < 0) return fail(GPUQT_ERR_ARG, "M must be >= 0");
  if (M == 0) return GPUQT_OK;
  gpuqt_status st;
  if ((st = check_vec(phiL, "phiL")) || (st = check_vec(phiR, "phiR")) || (st = check_vec(mu, "mu")))
    return st;
  const WsLayout W = ws_layout(h, 4, B, moment_rows(M), 0);
  if (!ws || ws_bytes < W.total) return fail(GPUQT_ERR_WORKSPACE, "workspace too small");
  if (!aligned16(ws)) return fail(GPUQT_ERR_ARG, "workspace is not 16-byte aligned");
  if ((st = check_device(h))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  double2* A = reinterpret_cast<double2*>(base);
  double2* Bf = reinterpret_cast<double2*>(base + W.vec_bytes);
  double2* part = reinterpret_cast<double2*>(base + W.off_part);
  if ((st = run_moments(h, B, reinterpret_cast<const double2*>(phiL), reinterpret_cast<const double2*>(phiR), M,
                        part, A, Bf, s)))
    return st;
  HIP_TRY(launch_reduce_moments(part, M, h->G_of(B, FAM_MOMENT), B, h->n_seg, h->blk0_of(B, FAM_MOMENT), 0,
                                reinterpret_cast<double2*>(mu), nullptr, s));
  return GPUQT_OK;
}

gpuqt_status gpuqt_evolve(gpuqt_h hh, int32_t B, double dt, int32_t Np, const double* psi_in,
                          double* psi_out, const double* chi_in, double* chi_out, void* ws,
                          size_t ws_bytes, void* stream) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  if (!std::isfinite(dt)) return fail(GPUQT_ERR_ARG, "dt is not finite");
  if (Np < 0) return fail(GPUQT_ERR_ARG, "Np must be >= 0");
  gpuqt_status st;
  if ((st = check_vec(psi_in, "psi_in")) || (st = check_vec(psi_out, "psi_out"))) return st;
  if (chi_in && !aligned16(chi_in)) return fail(GPUQT_ERR_ARG, "chi_in is not 16-byte aligned");
  if (chi_out && !aligned16(chi_out)) return fail(GPUQT_ERR_ARG, "chi_out is not 16-byte aligned");
  if (chi_in && !chi_out) return fail(GPUQT_ERR_ARG, "chi_in given without chi_out");
  const size_t vb = (size_t)h->n * B * 16;
  if (overlap(psi_out, psi_in, vb) || overlap(psi_out, chi_in, vb) || overlap(chi_out, psi_in, vb) ||
      overlap(chi_out, chi_in, vb) || overlap(chi_out, psi_out, vb))
    return fail(GPUQT_ERR_ARG, "outputs of gpuqt_evolve must not overlap its inputs or each other");
  const int np = terms_for(h, dt, Np);
  if (np < 1) return fail(GPUQT_ERR_ARG, "could not choose the number of terms");
  const int op = chi_out ? GPUQT_OP_EVOLVE_COMMUTATOR : GPUQT_OP_EVOLVE;
  const WsLayout W = ws_layout(h, op_vectors(op), B, 0, np);
  if (!ws || ws_bytes < W.total) return fail(GPUQT_ERR_WORKSPACE, "workspace too small");
  if (!aligned16(ws)) return fail(GPUQT_ERR_ARG, "workspace is not 16-byte aligned");
  if ((st = check_device(h))) return st;
  char* base = static_cast<char*>(ws);
  auto V = [&](int i) { return reinterpret_cast<double2*>(base + W.vec_bytes * i); };
  double* J = reinterpret_cast<double*>(base + W.off_J);
  return run_evolve(h, B, dt, np, reinterpret_cast<const double2*>(psi_in),
                    reinterpret_cast<double2*>(psi_out), reinterpret_cast<const double2*>(chi_in),
                    reinterpret_cast<double2*>(chi_out), V(0), V(1), chi_out ? V(2) : nullptr,
                    chi_out ? V(3) : nullptr, chi_out ? V(4) : nullptr, J,
                    static_cast<hipStream_t>(stream));
}

gpuqt_status gpuqt_apply_commutator(gpuqt_h hh, int32_t B, int32_t which, const double* psi,
                                    double* out, void* stream) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  if (which != GPUQT_VELOCITY && which != GPUQT_COMMUTATOR_XH)
    return fail(GPUQT_ERR_ARG, "which must be GPUQT_VELOCITY or GPUQT_COMMUTATOR_XH");
  gpuqt_status st;
  if ((st = check_vec(psi, "psi")) || (st = check_vec(out, "out"))) return st;
  if (overlap(psi, out, (size_t)h->n * B * 16)) return fail(GPUQT_ERR_ARG, "psi and out overlap");
  if ((st = check_device(h))) return st;
  HIP_TRY(launch_commutator(h->view(B), h->hop_mode, B, which, reinterpret_cast<const double2*>(psi),
                            reinterpret_cast<double2*>(out), static_cast<hipStream_t>(stream)));
  return GPUQT_OK;
}

static gpuqt_status check_series(const Handle* h, int32_t B, const double* phi, int32_t n_t,
                                 const double* dt, int32_t M, int32_t Np, const double* out) {
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  if (n_t < 0 || M < 0 || Np < 0) return fail(GPUQT_ERR_ARG, "n_t, M and Np must be >= 0");
  if (n_t > 0 && !dt) return fail(GPUQT_ERR_ARG, "dt is NULL");
  for (int k = 0; k < n_t; ++k)
    if (!std::isfinite(dt[k])) return fail(GPUQT_ERR_ARG, "dt contains a non-finite value");
  gpuqt_status st;
  if ((st = check_vec(phi, "phi"))) return st;
  if (!out) return fail(GPUQT_ERR_ARG, "out is NULL");
  return GPUQT_OK;
}

static int max_terms(const Handle* h, int32_t n_t, const double* dt, int32_t Np) {
  int best = 1;
  for (int k = 0; k < n_t; ++k) best = std::max(best, terms_for(h, dt[k], Np));
  return best;
}

// Recorded VAC forward ("tape"), for a backward pass that recomputes nothing:
// vector slots of n x B complex128 (256-byte aligned) holding psi_L(k) for
// k = 1 .. n_t-1 (slot k-1), psi_R(k) for k = 0 .. n_t-1 (slot n_t-1+k),
// for each row k from slot 2 n_t - 1 + 2 K k the two moment chains a_1..a_K,
// b_1..b_K of <V psi_L(k)| T_n |psi_R(k)> (K = max(1, M/2)), and for each
// time step k < n_t - 1 the two evolution chains T_m psi_L(k), T_m psi_R(k),
// m = 1 .. P-1, in 2 (P - 1) slots, P the largest number of terms of the steps.
static int64_t vac_tape_vectors(int n_t, int M, int P) {
  return n_t > 0 ? 2 * (int64_t)n_t - 1 + 2 * (int64_t)pair_steps(M) * n_t +
                       2 * (int64_t)std::max(P - 1, 0) * (n_t - 1)
                 : 0;
}

struct VacTape {
  char* base = nullptr;
  size_t vec_bytes = 0;
  int n_t = 0, K = 0, P = 1;
  double2* slot(int64_t i) const { return reinterpret_cast<double2*>(base + vec_bytes * (size_t)i); }
  double2* psiL(int k) const { return slot(k - 1); }
  double2* psiR(int k) const { return slot(n_t - 1 + k); }
  // a_1..a_K, b_1..b_K of row k
  std::vector<double2*> chains(int k) const {
    std::vector<double2*> c(2 * (size_t)K);
    for (int j = 0; j < 2 * K; ++j) c[j] = slot(2 * (int64_t)n_t - 1 + 2 * (int64_t)K * k + j);
    return c;
  }
  // time step k with np terms: T_m psi_L(k) at [m-1], T_m psi_R(k) at [np-1+m-1]
  std::vector<double2*> evolution(int k, int np) const {
    const int64_t base_k = 2 * (int64_t)n_t - 1 + 2 * (int64_t)K * n_t + 2 * (int64_t)(P - 1) * k;
    std::vector<double2*> c(2 * (size_t)std::max(np - 1, 0));
    for (int j = 0; j < np - 1; ++j) {
      c[j] = slot(base_k + j);
      c[np - 1 + j] = slot(base_k + (P - 1) + j);
    }
    return c;
  }
};

static gpuqt_status vac_tape_check(const Handle* h, int B, int n_t, int M, int P, void* tape,
                                   size_t tape_bytes, VacTape* T) {
  T->vec_bytes = round_up((size_t)h->n * (size_t)B * 16u, 256);
  T->n_t = n_t;
  T->K = pair_steps(M);
  T->P = P;
  T->base = static_cast<char*>(tape);
  if (!tape || tape_bytes < T->vec_bytes * (size_t)vac_tape_vectors(n_t, M, P))
    return fail(GPUQT_ERR_WORKSPACE, "tape too small");
  if (!aligned16(tape)) return fail(GPUQT_ERR_ARG, "tape is not 16-byte aligned");
  return GPUQT_OK;
}

static gpuqt_status vac_impl(const Handle* h, int32_t B, const double* phi, int32_t n_t, const double* dt, int32_t M,
                      int32_t Np, double* out, void* ws, size_t ws_bytes, void* tape, size_t tape_bytes,
                      void* stream) {
  gpuqt_status st = check_series(h, B, phi, n_t, dt, M, Np, out);
  if (st) return st;
  if (n_t == 0 || M == 0) return GPUQT_OK;
  const int np = max_terms(h, n_t - 1, dt, Np);
  VacTape T;
  if (tape && (st = vac_tape_check(h, B, n_t, M, np, tape, tape_bytes, &T))) return st;
  const WsLayout W = ws_layout(h, op_vectors(GPUQT_OP_VAC), B, moment_rows(M), np);
  if (!ws || ws_bytes < W.total) return fail(GPUQT_ERR_WORKSPACE, "workspace too small");
  if (!aligned16(ws)) return fail(GPUQT_ERR_ARG, "workspace is not 16-byte aligned");
  if ((st = check_device(h))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  auto V = [&](int i) { return reinterpret_cast<double2*>(base + W.vec_bytes * i); };
  double2* part = reinterpret_cast<double2*>(base + W.off_part);
  double* J = reinterpret_cast<double*>(base + W.off_J);
  const DevMat D = h->view(B);
  // psi_L = phi (input, read only), psi_R = V phi
  const double2* psiL = reinterpret_cast<const double2*>(phi);
  double2* Lbuf[2] = {V(0), V(1)};
  double2* Rbuf[2] = {V(2), V(3)};
  double2* phiL = V(4);
  int ri = 0;
  HIP_TRY(launch_commutator(D, h->hop_mode, B, GPUQT_VELOCITY, psiL, tape ? T.psiR(0) : Rbuf[0], s));
  const double2* psiR = tape ? T.psiR(0) : Rbuf[0];
  const int64_t row = (int64_t)h->n_seg * B * M;
  for (int k = 0; k < n_t; ++k) {
    HIP_TRY(launch_commutator(D, h->hop_mode, B, GPUQT_VELOCITY, psiL, phiL, s));
    if (tape) {
      const std::vector<double2*> keep = T.chains(k);
      if ((st = run_moments(h, B, phiL, psiR, M, part, nullptr, nullptr, s, false, nullptr, nullptr,
                            keep.data())))
        return st;
    } else if ((st = run_moments(h, B, phiL, psiR, M, part, V(5), V(6), s, false, V(7), V(8)))) {
      return st;
    }
    HIP_TRY(launch_reduce_moments(part, M, h->G_of(B, FAM_PAIR), B, h->n_seg, h->blk0_of(B, FAM_PAIR), 1,
                                  nullptr, out + row * k, s));
    if (k + 1 < n_t) {
      const int np_k = terms_for(h, dt[k], Np);
      double2* Ln = tape ? T.psiL(k + 1) : (psiL == Lbuf[0]) ? Lbuf[1] : Lbuf[0];
      double2* Rn = tape ? T.psiR(k + 1) : Rbuf[ri ^ 1];
      // both states advance with the same U(-dt): one two-chain series
      const std::vector<double2*> ev = tape ? T.evolution(k, np_k) : std::vector<double2*>();
      if ((st = run_evolve_pair(h, B, -dt[k], np_k, psiL, Ln, psiR, Rn, V(5), V(6), V(7), V(8), J, s,
                                tape ? ev.data() : nullptr)))
        return st;
      psiL = Ln;
      psiR = Rn;
      ri ^= 1;
    }
  }
  return GPUQT_OK;
}

gpuqt_status gpuqt_vac(gpuqt_h hh, int32_t B, const double* phi, int32_t n_t, const double* dt,
                       int32_t M, int32_t Np, double* out, void* ws, size_t ws_bytes, void* stream) {
  return vac_impl(reinterpret_cast<const Handle*>(hh), B, phi, n_t, dt, M, Np, out, ws, ws_bytes, nullptr, 0,
                  stream);
}

gpuqt_status gpuqt_vac_tape_size(gpuqt_h hh, int32_t B, int32_t n_t, const double* dt, int32_t M, int32_t Np,
                                 size_t* bytes) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h || !bytes) return fail(GPUQT_ERR_ARG, "NULL handle or bytes");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  if (n_t < 0 || M < 0 || Np < 0) return fail(GPUQT_ERR_ARG, "n_t, M and Np must be >= 0");
  if (n_t > 1 && !dt) return fail(GPUQT_ERR_ARG, "dt is NULL");
  const int np = n_t > 1 ? max_terms(h, n_t - 1, dt, Np) : 1;
  *bytes = round_up((size_t)h->n * (size_t)B * 16u, 256) * (size_t)vac_tape_vectors(n_t, M, np);
  return GPUQT_OK;
}

gpuqt_status gpuqt_vac_record(gpuqt_h hh, int32_t B, const double* phi, int32_t n_t, const double* dt,
                              int32_t M, int32_t Np, double* out, void* ws, size_t ws_bytes, void* tape,
                              size_t tape_bytes, void* stream) {
  if (!tape) return fail(GPUQT_ERR_ARG, "tape is NULL");
  return vac_impl(reinterpret_cast<const Handle*>(hh), B, phi, n_t, dt, M, Np, out, ws, ws_bytes, tape,
                  tape_bytes, stream);
}

gpuqt_status gpuqt_msd(gpuqt_h hh, int32_t B, const double* phi, int32_t n_t, const double* dt,
                       int32_t M, int32_t Np, double* out, void* ws, size_t ws_bytes, void* stream) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  gpuqt_status st = check_series(h, B, phi, n_t, dt, M, Np, out);
  if (st) return st;
  if (n_t == 0 || M == 0) return GPUQT_OK;
  const int np = max_terms(h, n_t, dt, Np);
  const WsLayout W = ws_layout(h, op_vectors(GPUQT_OP_MSD), B, moment_rows(M), np);
  if (!ws || ws_bytes < W.total) return fail(GPUQT_ERR_WORKSPACE, "workspace too small");
  if (!aligned16(ws)) return fail(GPUQT_ERR_ARG, "workspace is not 16-byte aligned");
  if ((st = check_device(h))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  auto V = [&](int i) { return reinterpret_cast<double2*>(base + W.vec_bytes * i); };
  double2* part = reinterpret_cast<double2*>(base + W.off_part);
  double* J = reinterpret_cast<double*>(base + W.off_J);
  double2* Pbuf[2] = {V(0), V(1)};
  double2* Cbuf[2] = {V(2), V(3)};
  const double2* psi = reinterpret_cast<const double2*>(phi);
  const double2* chi = nullptr;
  int pi = 0;
  const int64_t row = (int64_t)h->n_seg * B * M;
  for (int k = 0; k < n_t; ++k) {
    const int np_k = terms_for(h, dt[k], Np);
    double2* Pn = Pbuf[pi];
    double2* Cn = Cbuf[pi];
    if ((st = run_evolve(h, B, dt[k], np_k, psi, Pn, chi, Cn, V(4), V(5), V(6), V(7), V(8), J, s)))
      return st;
    if ((st = run_moments(h, B, Cn, Cn, M, part, V(4), V(5), s, true))) return st;
    HIP_TRY(launch_reduce_moments(part, M, h->G_of(B, FAM_SYM), B, h->n_seg, h->blk0_of(B, FAM_SYM), 1,
                                  nullptr, out + row * k, s));
    psi = Pn;
    chi = Cn;
    pi ^= 1;
  }
  return GPUQT_OK;
}

gpuqt_status gpuqt_moments_backward(gpuqt_h hh, int32_t B, const double* phiL, const double* phiR,
                                    int32_t M, const double* w, double* grad_onsite,
                                    double* grad_class, double* grad_hop, double* lam0,
                                    int32_t ckpt_stride, void* ws, size_t ws_bytes, void* stream) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  if (M < 0 || ckpt_stride < 0) return fail(GPUQT_ERR_ARG, "M and ckpt_stride must be >= 0");
  if (M == 0) return GPUQT_OK;
  gpuqt_status st;
  if ((st = check_vec(phiL, "phiL")) || (st = check_vec(phiR, "phiR"))) return st;
  if (!w) return fail(GPUQT_ERR_ARG, "w is NULL");
  if (!grad_onsite && (grad_class || grad_hop))
    return fail(GPUQT_ERR_ARG, "grad_class and grad_hop need grad_onsite");
  if (grad_hop && (reinterpret_cast<uintptr_t>(grad_hop) & 7u))
    return fail(GPUQT_ERR_ARG, "grad_hop is not 8-byte aligned");
  if (lam0 && !aligned16(lam0)) return fail(GPUQT_ERR_ARG, "lam0 is not 16-byte aligned");
  if (grad_class && h->n_class > 4)
    return fail(GPUQT_ERR_UNSUPPORTED, "class gradients support at most 4 hopping classes");
  const int s = backward_stride(M, ckpt_stride);
  const WsLayout W = ws_layout(h, backward_vectors(M, s), B, s == 1 ? 5 : 2, s == 1 ? raw_weight_len(B, M) : 0);
  if (!ws || ws_bytes < W.total) return fail(GPUQT_ERR_WORKSPACE, "workspace too small");
  if (!aligned16(ws)) return fail(GPUQT_ERR_ARG, "workspace is not 16-byte aligned");
  if ((st = check_device(h))) return st;
  hipStream_t sm = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  std::vector<double2*> vec(backward_vectors(M, s));
  for (size_t i = 0; i < vec.size(); ++i) vec[i] = reinterpret_cast<double2*>(base + W.vec_bytes * i);
  double* gcp = reinterpret_cast<double*>(base + W.off_part);
  const int nc = grad_class ? class_stride(h->n_class) : 0;
  if (nc) HIP_TRY(launch_zero(gcp, (int64_t)h->G * nc, sm));
  // per-entry gradients: the reverse of the plain recurrence (the product-identity
  // forms use H^+ = H, which an entry on its own does not keep)
  if (s == 1 && !grad_hop && phiL == phiR) {   // Hermitian set, every vector kept: one-chain reverse
    if ((st = run_backward_sym(h, B, reinterpret_cast<const double2*>(phiL), M, w, grad_onsite, gcp, nc,
                               reinterpret_cast<double2*>(lam0), false, vec.data(),
                               reinterpret_cast<double*>(base + W.off_J),
                               reinterpret_cast<double2*>(base + W.off_part) + 2 * (int64_t)h->G * B, sm)))
      return st;
  } else if (s == 1 && !grad_hop) {   // every forward vector kept: reverse of the two-chain form
    if ((st = run_backward_pair(h, B, reinterpret_cast<const double2*>(phiL),
                                reinterpret_cast<const double2*>(phiR), M, w, grad_onsite, gcp, nc,
                                nullptr, false, reinterpret_cast<double2*>(lam0), false, vec.data(),
                                reinterpret_cast<double*>(base + W.off_J),
                                reinterpret_cast<double2*>(base + W.off_part) + 2 * (int64_t)h->G * B, sm)))
      return st;
  } else {
    BwdSource src;
    src.wts = w;
    if ((st = run_backward(h, B, reinterpret_cast<const double2*>(phiL),
                           reinterpret_cast<const double2*>(phiR), M, src, grad_onsite, gcp, nc,
                           reinterpret_cast<double2*>(lam0), false, s, vec.data(), sm, nullptr, grad_hop)))
      return st;
  }
  if (nc) HIP_TRY(launch_reduce_classes(gcp, h->G, nc, h->n_class, grad_class, sm));
  return GPUQT_OK;
}

// Time checkpoints of the VAC adjoint: stride 1 keeps every state
// psi_{L,R}(t_k); s >= 2 keeps the states of rows 0, s, 2s, ... and
// re-evolves one segment of s rows at a time during the reverse pass; 0
// chooses ceil(sqrt(n_t)).
static int vac_time_stride(int n_t, int time_stride) {
  if (time_stride >= 1) return std::min(time_stride, std::max(n_t, 1));
  const int st = (int)std::ceil(std::sqrt((double)std::max(n_t, 1)));
  return st >= n_t ? 1 : std::max(2, st);
}

// state vectors the forward part of gpuqt_vac_backward keeps: every psi_L(k)
// (k >= 1) and psi_R(k) at stride 1; else the checkpoints (psi_L of row 0 is
// phi itself) and the s - 1 later states of one segment per chain
static int vac_state_vectors(int n_t, int ts) {
  if (ts <= 1) return 2 * n_t - 1;
  const int nck = (n_t + ts - 1) / ts;
  return 2 * nck - 1 + 2 * (ts - 1);
}

// number of workspace vectors of gpuqt_vac_backward (keep: every forward vector
// kept, two-chain reverse of the rows; else checkpoints every ceil(sqrt(L)) steps)
static int vac_backward_vectors(int n_t, int M, int Np, bool keep, int ts) {
  const int L = std::max(M, Np);
  return vac_state_vectors(n_t, ts) + 6 + backward_vectors(L, keep ? 1 : backward_stride(L, 0));
}

gpuqt_status gpuqt_vac_backward_workspace_size(gpuqt_h hh, int32_t B, int32_t n_t, const double* dt,
                                               int32_t M, int32_t Np, int32_t ckpt_stride, int32_t time_stride,
                                               size_t* bytes) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h || !bytes) return fail(GPUQT_ERR_ARG, "NULL handle or bytes");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  if (n_t < 0 || M < 0 || Np < 0 || (n_t > 0 && !dt)) return fail(GPUQT_ERR_ARG, "bad sizes");
  if (ckpt_stride != 0 && ckpt_stride != 1) return fail(GPUQT_ERR_ARG, "ckpt_stride must be 0 or 1");
  if (time_stride < 0) return fail(GPUQT_ERR_ARG, "time_stride must be >= 0");
  const bool keep = ckpt_stride == 1;
  const int np = max_terms(h, std::max(n_t - 1, 0), dt, Np);
  *bytes = ws_layout(h, vac_backward_vectors(n_t, M, np, keep, vac_time_stride(n_t, time_stride)), B, keep ? 5 : 2,
                     np + (keep ? raw_weight_len(B, M) : 0)).total;
  return GPUQT_OK;
}

static gpuqt_status vac_backward_impl(const Handle* h, int32_t B, const double* phi, int32_t n_t,
                                      const double* dt, int32_t M, int32_t Np, const double* w,
                                      double* grad_onsite, double* grad_class, double* grad_hop,
                                      int32_t ckpt_stride, int32_t time_stride, void* tape, size_t tape_bytes,
                                      void* ws, size_t ws_bytes, void* stream) {
  gpuqt_status st = check_series(h, B, phi, n_t, dt, M, Np, w);
  if (st) return st;
  if (ckpt_stride != 0 && ckpt_stride != 1) return fail(GPUQT_ERR_ARG, "ckpt_stride must be 0 or 1");
  if (time_stride < 0) return fail(GPUQT_ERR_ARG, "time_stride must be >= 0");
  const bool keep = ckpt_stride == 1 || tape;
  if (!grad_onsite) return fail(GPUQT_ERR_ARG, "grad_onsite is NULL");
  if (grad_hop && (reinterpret_cast<uintptr_t>(grad_hop) & 7u))
    return fail(GPUQT_ERR_ARG, "grad_hop is not 8-byte aligned");
  if (grad_class && h->n_class > 4)
    return fail(GPUQT_ERR_UNSUPPORTED, "class gradients support at most 4 hopping classes");
  if (n_t == 0 || M == 0) return GPUQT_OK;
  const int np = max_terms(h, n_t - 1, dt, Np);
  VacTape T;
  if (tape && (st = vac_tape_check(h, B, n_t, M, np, tape, tape_bytes, &T))) return st;
  const int L = tape ? np : std::max(M, np);
  const int s = keep ? 1 : backward_stride(L, 0);
  const int ts = tape ? 1 : vac_time_stride(n_t, time_stride);
  const int nv = tape ? 6 + backward_vectors(np, 1) : vac_backward_vectors(n_t, M, np, keep, ts);
  const WsLayout W = ws_layout(h, nv, B, keep ? 5 : 2, np + (keep ? raw_weight_len(B, M) : 0));
  if (!ws || ws_bytes < W.total) return fail(GPUQT_ERR_WORKSPACE, "workspace too small");
  if (!aligned16(ws)) return fail(GPUQT_ERR_ARG, "workspace is not 16-byte aligned");
  if ((st = check_device(h))) return st;
  hipStream_t sm = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  auto V = [&](int i) { return reinterpret_cast<double2*>(base + W.vec_bytes * i); };
  double* gcp = reinterpret_cast<double*>(base + W.off_part);
  double* J = reinterpret_cast<double*>(base + W.off_J);
  const DevMat D = h->view(B);
  const int nc = grad_class ? class_stride(h->n_class) : 0;
  const double2* ph = reinterpret_cast<const double2*>(phi);
  // states: the recorded tape; every psi_L(k) (k >= 1) and psi_R(k); or (time
  // checkpoints) psi_L, psi_R of rows 0, ts, 2 ts, ... and the states of one
  // segment of ts rows, re-evolved from its checkpoint when the reverse needs it
  const int o = tape ? 0 : vac_state_vectors(n_t, ts);
  const int nck = ts > 1 ? (n_t + ts - 1) / ts : 0;
  auto ckL = [&](int c) -> const double2* { return c == 0 ? ph : V(c - 1); };      // checkpoint c, chain L
  auto ckR = [&](int c) -> double2* { return V(nck - 1 + c); };                    // checkpoint c, chain R
  auto segL = [&](int i) -> double2* { return V(2 * nck - 1 + (i - 1)); };          // i = 1 .. ts-1
  auto segR = [&](int i) -> double2* { return V(2 * nck - 1 + (ts - 1) + (i - 1)); };
  int seg = -1;   // the segment whose states segL / segR hold (time checkpoints)
  auto psiL = [&](int k) -> const double2* {
    if (k == 0) return ph;
    if (tape) return T.psiL(k);
    if (ts <= 1) return V(k - 1);
    const int i = k - seg * ts;
    return i == 0 ? ckL(seg) : segL(i);
  };
  auto psiR = [&](int k) -> double2* {
    if (tape) return T.psiR(k);
    if (ts <= 1) return V(n_t - 1 + k);
    const int i = k - seg * ts;
    return i == 0 ? ckR(seg) : segR(i);
  };
  double2* gL[2] = {V(o), V(o + 1)};
  double2* gR[2] = {V(o + 2), V(o + 3)};
  double2* gphiL = V(o + 4);
  double2* phiL = V(o + 5);
  std::vector<double2*> pool(backward_vectors(L, s));
  for (size_t i = 0; i < pool.size(); ++i) pool[i] = V(o + 6 + (int)i);
  double2* e0 = pool[0];   // evolution scratch (forward pass and segment re-evolution)
  double2* e1 = pool[1];
  if (nc) HIP_TRY(launch_zero(gcp, (int64_t)h->G * nc, sm));
  // states of segment c from its checkpoint: psi(k+1) = U(-dt_k) psi(k), k in the segment
  auto load_segment = [&](int c) -> gpuqt_status {
    seg = c;
    const int k0 = c * ts, k1 = std::min(k0 + ts, n_t);
    for (int k = k0; k + 1 < k1; ++k) {
      const int i = k - k0;
      gpuqt_status q = run_evolve_pair(h, B, -dt[k], terms_for(h, dt[k], Np), i == 0 ? ckL(c) : segL(i), segL(i + 1),
                                       i == 0 ? ckR(c) : segR(i), segR(i + 1), e0, e1, pool[2], pool[3], J, sm);
      if (q) return q;
    }
    return GPUQT_OK;
  };
  // forward (unless recorded): psi_R(0) = V phi; psi_{L,R}(k+1) = U(-dt_k) psi_{L,R}(k)
  if (!tape && ts <= 1) {
    HIP_TRY(launch_commutator(D, h->hop_mode, B, GPUQT_VELOCITY, ph, psiR(0), sm));
    for (int k = 0; k + 1 < n_t; ++k) {
      const int npk = terms_for(h, dt[k], Np);
      if ((st = run_evolve_pair(h, B, -dt[k], npk, psiL(k), V(k), psiR(k), psiR(k + 1), e0, e1, pool[2],
                                pool[3], J, sm)))
        return st;
    }
  } else if (!tape) {
    // keep only the checkpoints; a state between checkpoints goes to segment
    // slot 1 or 2 by the parity of its row (ts >= 3), or to slot 1 (ts = 2,
    // where it always follows a checkpoint), so it never overwrites its input
    HIP_TRY(launch_commutator(D, h->hop_mode, B, GPUQT_VELOCITY, ph, ckR(0), sm));
    const double2* aL = ph;
    const double2* aR = ckR(0);
    for (int k = 0; k + 1 < n_t; ++k) {
      const int npk = terms_for(h, dt[k], Np);
      double2* oL;
      double2* oR;
      if ((k + 1) % ts == 0) {
        oL = const_cast<double2*>(ckL((k + 1) / ts));
        oR = ckR((k + 1) / ts);
      } else {
        const int slot = ts >= 3 ? ((k + 1) % 2) + 1 : 1;
        oL = segL(slot);
        oR = segR(slot);
      }
      if ((st = run_evolve_pair(h, B, -dt[k], npk, aL, oL, aR, oR, e0, e1, pool[2], pool[3], J, sm))) return st;
      aL = oL;
      aR = oR;
    }
  }
  // reverse over the rows
  int cl = 0, cr = 0;
  HIP_TRY(launch_scale(D, B, nullptr, gL[0], nullptr, 0, sm));
  HIP_TRY(launch_scale(D, B, nullptr, gR[0], nullptr, 0, sm));
  const int64_t row = (int64_t)h->n_seg * B * M;
  if (!tape && ts > 1 && (st = load_segment((n_t - 1) / ts))) return st;
  for (int k = n_t - 1; k >= 0; --k) {
    HIP_TRY(launch_commutator(D, h->hop_mode, B, GPUQT_VELOCITY, psiL(k), phiL, sm));
    if (keep && !grad_hop) {
      // moments of row k by the two-chain reverse: parameter terms,
      // gphiL = sum_n w_n T_n psi_R(k) and gR += sum_n w_n T_n phiL in one pass
      const std::vector<double2*> rec = tape ? T.chains(k) : std::vector<double2*>();
      if ((st = run_backward_pair(h, B, phiL, psiR(k), M, w + row * k, grad_onsite, gcp, nc, gphiL, false,
                                  gR[cr], true, pool.data(), J + (int64_t)h->n_seg * np,
                                  reinterpret_cast<double2*>(base + W.off_part) + 2 * (int64_t)h->G * B, sm,
                                  tape ? rec.data() : nullptr)))
        return st;
    } else {
      BwdSource src;
      src.wts = w + row * k;
      // moments of row k: parameter terms, and gR += sum_n w_n T_n phiL (with
      // per-entry gradients also when every vector is kept: the plain
      // recurrence, not the two-chain form, whose pool it fits)
      if ((st = run_backward(h, B, phiL, psiR(k), M, src, grad_onsite, gcp, nc, gR[cr], true, s,
                             pool.data(), sm, nullptr, grad_hop)))
        return st;
      // gphiL = sum_n w_n T_n psi_R(k) (no parameter terms)
      if ((st = run_backward(h, B, psiR(k), phiL, M, src, nullptr, nullptr, 0, gphiL, false, s,
                             pool.data(), sm)))
        return st;
    }
    // phiL = V psi_L: gL += V gphiL, class terms of V
    HIP_TRY(launch_commutator(D, h->hop_mode, B, GPUQT_VELOCITY | kAccumulate, gphiL, gL[cl], sm));
    if (nc) HIP_TRY(launch_velocity_class_grad(D, h->hop_mode, B, nc, gphiL, psiL(k), h->d_cls, gcp, sm));
    if (grad_hop)
      HIP_TRY(launch_velocity_entry_grad(D, h->hop_mode, B, gphiL, psiL(k), grad_hop, h->max_nn_in, sm));
    if (k == 0) break;
    // the reverse through U(-dt_{k-1}) needs the states of row k - 1
    if (!tape && ts > 1 && (k - 1) / ts != seg && (st = load_segment((k - 1) / ts))) return st;
    // back through psi(k) = U(-dt) psi(k-1): parameter terms and g <- U(+dt) g
    const double d = -dt[k - 1];
    const int npk = terms_for(h, d, Np);
    HIP_TRY(launch_bessel_table(h->d_seg_dE, h->n_seg, std::fabs(d), npk, npk, J, sm));
    BwdSource ev;
    ev.Jtab = J;
    ev.ldJ = npk;
    ev.sgn = d >= 0 ? 1.0 : -1.0;
    // the chains T_m psi_{L,R}(k-1) were recorded by the forward's evolution
    const std::vector<double2*> rec = tape ? T.evolution(k - 1, npk) : std::vector<double2*>();
    const bool have = tape && npk >= 3;
    if ((st = run_backward(h, B, gL[cl], psiL(k - 1), npk, ev, grad_onsite, gcp, nc, gL[cl ^ 1], false,
                           s, pool.data(), sm, have ? rec.data() : nullptr, grad_hop)))
      return st;
    if ((st = run_backward(h, B, gR[cr], psiR(k - 1), npk, ev, grad_onsite, gcp, nc, gR[cr ^ 1], false,
                           s, pool.data(), sm, have ? rec.data() + (npk - 1) : nullptr, grad_hop)))
      return st;
    cl ^= 1;
    cr ^= 1;
  }
  // psi_R(0) = V phi: class terms of V
  if (nc) HIP_TRY(launch_velocity_class_grad(D, h->hop_mode, B, nc, gR[cr], ph, h->d_cls, gcp, sm));
  if (grad_hop) HIP_TRY(launch_velocity_entry_grad(D, h->hop_mode, B, gR[cr], ph, grad_hop, h->max_nn_in, sm));
  if (nc) HIP_TRY(launch_reduce_classes(gcp, h->G, nc, h->n_class, grad_class, sm));
  return GPUQT_OK;
}

gpuqt_status gpuqt_vac_backward(gpuqt_h hh, int32_t B, const double* phi, int32_t n_t,
                                const double* dt, int32_t M, int32_t Np, const double* w,
                                double* grad_onsite, double* grad_class, double* grad_hop, int32_t ckpt_stride,
                                int32_t time_stride, void* ws, size_t ws_bytes, void* stream) {
  return vac_backward_impl(reinterpret_cast<const Handle*>(hh), B, phi, n_t, dt, M, Np, w, grad_onsite,
                           grad_class, grad_hop, ckpt_stride, time_stride, nullptr, 0, ws, ws_bytes, stream);
}

gpuqt_status gpuqt_tie_entry_gradient(gpuqt_h hh, const double* untied, double* tied, void* stream) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (!untied || !tied) return fail(GPUQT_ERR_ARG, "untied or tied is NULL");
  if (untied == tied) return fail(GPUQT_ERR_ARG, "untied and tied must be distinct buffers");
  if ((reinterpret_cast<uintptr_t>(untied) & 7u) || (reinterpret_cast<uintptr_t>(tied) & 7u))
    return fail(GPUQT_ERR_ARG, "untied or tied is not 8-byte aligned");
  gpuqt_status st;
  if ((st = check_device(h))) return st;
  HIP_TRY(launch_tie_entries(h->view(1), h->hop_mode, h->n, h->max_nn_in, untied, tied,
                             static_cast<hipStream_t>(stream)));
  return GPUQT_OK;
}

gpuqt_status gpuqt_vac_backward_tape_workspace_size(gpuqt_h hh, int32_t B, int32_t n_t, const double* dt,
                                                    int32_t M, int32_t Np, size_t* bytes) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h || !bytes) return fail(GPUQT_ERR_ARG, "NULL handle or bytes");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  if (n_t < 0 || M < 0 || Np < 0 || (n_t > 0 && !dt)) return fail(GPUQT_ERR_ARG, "bad sizes");
  const int np = max_terms(h, std::max(n_t - 1, 0), dt, Np);
  *bytes = ws_layout(h, 6 + backward_vectors(np, 1), B, 5, np + raw_weight_len(B, M)).total;
  return GPUQT_OK;
}

gpuqt_status gpuqt_vac_backward_tape(gpuqt_h hh, int32_t B, const double* phi, int32_t n_t, const double* dt,
                                     int32_t M, int32_t Np, const double* w, double* grad_onsite,
                                     double* grad_class, const void* tape, size_t tape_bytes, void* ws,
                                     size_t ws_bytes, void* stream) {
  if (!tape) return fail(GPUQT_ERR_ARG, "tape is NULL");
  return vac_backward_impl(reinterpret_cast<const Handle*>(hh), B, phi, n_t, dt, M, Np, w, grad_onsite,
                           grad_class, nullptr, 1, 1, const_cast<void*>(tape), tape_bytes, ws, ws_bytes, stream);
}

gpuqt_status gpuqt_autotune(gpuqt_h hh, int32_t B, void* ws, size_t ws_bytes, void* stream,
                            double* times_us) {
  Handle* h = reinterpret_cast<Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (!valid_B(B)) return fail(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  constexpr int kSteps = kTuneSteps;
  const WsLayout W = ws_layout(h, 3, B, kSteps + 1, 0);
  if (!ws || ws_bytes < W.total) return fail(GPUQT_ERR_WORKSPACE, "workspace too small");
  if (!aligned16(ws)) return fail(GPUQT_ERR_ARG, "workspace is not 16-byte aligned");
  gpuqt_status st;
  if ((st = check_device(h))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  double2* phi = reinterpret_cast<double2*>(base);
  double2* A = reinterpret_cast<double2*>(base + W.vec_bytes);
  double2* Bf = reinterpret_cast<double2*>(base + 2 * W.vec_bytes);
  double2* part = reinterpret_cast<double2*>(base + W.off_part);
  // a unit-modulus start vector, like the random-phase vectors of the method
  HIP_TRY(launch_fill_phase(h->view(B), B, phi, s));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  // milliseconds of one run (after one untimed run of the same work)
  auto time_run = [&](auto&& run, float* ms) -> gpuqt_status {
    gpuqt_status q;
    if ((q = run())) return q;
    if (hipEventRecord(e0, s) != hipSuccess) return fail(GPUQT_ERR_HIP, "hipEventRecord failed");
    if ((q = run())) return q;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return fail(GPUQT_ERR_HIP, "event timing failed");
    return GPUQT_OK;
  };
  // the Hermitian moment step (the one most calls run) of one variant and cap
  // v: bit 0 non-temporal loads, bit 1 banded order, bit 2 the pencil order instead
  auto time_one = [&](int v, int cap, float* ms) -> gpuqt_status {
    h->nt = v & 1;
    h->banded = (v >> 1) & 1;
    h->pencil = (v >> 2) & 1;
    h->per_cu_cap = cap;
    return time_run([&] { return run_moments(h, B, phi, phi, kSteps + 1, part, A, Bf, s, true); }, ms);
  };
  const int lb = Handle::log2B(B);
  // caps below a family's occupancy limit at the current load variant, then none
  auto caps_of = [&](int fam, std::vector<int>* out) {
    const int occ = std::max<int>(1, h->occ[fam][lb][h->fam_nt(fam) ? 1 : 0]);
    out->clear();
    for (int cap : {2, 3, 4, 5, 6})
      if (cap < occ) out->push_back(cap);
    out->push_back(0);
  };
  for (int f = 0; f < kFamilies; ++f) h->fam_cap[f] = -1;
  h->series_nt_flip = 0;
  h->use_box = 0;
  h->use_box_msd = 0;
  float best = 0.0f;
  int best_v = (h->nt | (h->banded << 1) | ((h->banded & h->pencil) << 2)), best_cap = h->per_cu_cap;
  std::vector<int> vars = {0, 1};
  if (h->d_units[lb]) vars.insert(vars.end(), {2, 3});
  if (h->d_units_p[lb]) vars.insert(vars.end(), {6, 7});
  if (times_us)
    for (int v = 0; v < kTuneTimes; ++v) times_us[v] = 0.0;
  float ms = 0.0f;
  st = time_one(0, 0, &ms);   // settle clocks and caches before the sweep
  std::vector<int> caps;
  for (int v : vars) {
    if (st) break;
    h->nt = v & 1;
    caps_of(FAM_SYM, &caps);
    const int slot = v < 4 ? v : v - 2;   // times_us: 0..3 load/order variants, 4, 5 pencil
    for (int cap : caps) {
      if ((st = time_one(v, cap, &ms))) break;
      const double us = 1e3 * ms / (kSteps / 2);   // per launch
      if (times_us && (times_us[slot] == 0.0 || us < times_us[slot])) times_us[slot] = us;
      if (best == 0.0f || ms < best) {
        best = ms;
        best_v = v;
        best_cap = cap;
      }
    }
  }
  h->nt = best_v & 1;
  h->banded = (best_v >> 1) & 1;
  h->pencil = (best_v >> 2) & 1;
  h->per_cu_cap = best_cap;
  // on a periodic box (or segments that are all periodic squares: the sheet form), the
  // stencil kernel of the Hermitian step, uncapped and at
  // caps 1..6 (its loads run a plane ahead, so a few workgroups per CU fill HBM, and
  // fewer concurrent streams use the DRAM pages and the L2 better); when it beats the
  // best general variant it is kept, with its cap as the Hermitian family's own
  if (!st && (h->box[0] > 0 || h->sheet_ok) && B >= 2 && h->hop_mode == HOP_UNIFORM) {
    h->use_box = 1;
    float bbest = 0.0f;
    int bcap = 0;
    for (int cap : {0, 1, 2, 3, 4, 5, 6}) {
      h->fam_cap[FAM_SYM] = (int8_t)cap;
      float mb = 0.0f;
      if ((st = time_run([&] { return run_moments(h, B, phi, phi, kSteps + 1, part, A, Bf, s, true); }, &mb)))
        break;
      if (bbest == 0.0f || mb < bbest) {
        bbest = mb;
        bcap = cap;
      }
    }
    if (times_us && !st) times_us[kTuneTimes - 1] = 1e3 * bbest / (kSteps / 2);
    if (!st && bbest < best) {
      h->fam_cap[FAM_SYM] = (int8_t)bcap;
    } else {
      h->use_box = 0;
      h->fam_cap[FAM_SYM] = -1;
    }
  }
  // with room for their vectors, each of the two-chain moment, two-vector
  // evolution and MSD families also gets its own cap at this load variant
  const WsLayout WF = ws_layout(h, kTuneVectors, B, kSteps + 1, kTuneNp);
  if (!st && ws_bytes >= WF.total) {
    double2* v[kTuneVectors];
    for (int i = 0; i < kTuneVectors; ++i) v[i] = reinterpret_cast<double2*>(base + i * WF.vec_bytes);
    double2* partF = reinterpret_cast<double2*>(base + WF.off_part);
    double* J = reinterpret_cast<double*>(base + WF.off_J);
    HIP_TRY(launch_fill_phase(h->view(B), B, v[1], s));
    const double dt = 1.0;
    // one timed run of family f's kernels
    auto run_family = [&](int f) -> gpuqt_status {
      if (f == FAM_PAIR) return run_moments(h, B, v[0], v[1], kSteps + 1, partF, v[2], v[3], s, false, v[4], v[5]);
      if (f == FAM_EVOLVE_PAIR)
        return run_evolve_pair(h, B, dt, kTuneNp, v[0], v[2], v[1], v[3], v[4], v[5], v[6], v[7], J, s);
      return run_evolve(h, B, dt, kTuneNp, v[0], v[2], v[1], v[3], v[4], v[5], v[6], v[7], nullptr, J, s);
    };
    // the best cap of family f at the current load variants (its time in *best_ms)
    auto tune_family = [&](int f, float* best_ms) -> gpuqt_status {
      auto run = [&]() -> gpuqt_status { return run_family(f); };
      caps_of(f, &caps);
      float fbest = 0.0f;
      int fcap = -1;
      for (int cap : caps) {
        h->fam_cap[f] = (int8_t)cap;
        gpuqt_status q;
        if ((q = time_run(run, &ms))) return q;
        if (fbest == 0.0f || ms < fbest) {
          fbest = ms;
          fcap = cap;
        }
      }
      h->fam_cap[f] = (int8_t)fcap;
      *best_ms = fbest;
      return GPUQT_OK;
    };
    float t_pair = 0.0f;
    st = tune_family(FAM_PAIR, &t_pair);
    // the series families (two-vector evolution and MSD terms) with the handle's
    // load variant and with the other one; the pair of caps of the faster total stays
    float tot[2] = {0.0f, 0.0f}, tmsd[2] = {0.0f, 0.0f};
    int8_t cap_ev[2] = {-1, -1}, cap_msd[2] = {-1, -1};
    for (int flip = 0; flip < 2 && !st; ++flip) {
      h->series_nt_flip = flip;
      float te = 0.0f, tm = 0.0f;
      if ((st = tune_family(FAM_EVOLVE_PAIR, &te)) || (st = tune_family(FAM_MSD, &tm))) break;
      tot[flip] = te + tm;
      tmsd[flip] = tm;
      cap_ev[flip] = h->fam_cap[FAM_EVOLVE_PAIR];
      cap_msd[flip] = h->fam_cap[FAM_MSD];
    }
    if (!st) {
      const int fl = tot[1] < tot[0] ? 1 : 0;
      h->series_nt_flip = fl;
      h->fam_cap[FAM_EVOLVE_PAIR] = cap_ev[fl];
      h->fam_cap[FAM_MSD] = cap_msd[fl];
      // on a periodic box with uniform x steps, the MSD term's box stencil kernel,
      // uncapped and at caps 1..6, kept (with its cap) when faster
      if (h->box_msd_ok && B >= 2 && h->hop_mode == HOP_UNIFORM) {
        h->use_box_msd = 1;
        float bbest = 0.0f;
        int bcap = 0;
        for (int cap : {0, 1, 2, 3, 4, 5, 6}) {
          h->fam_cap[FAM_MSD] = (int8_t)cap;
          float mb = 0.0f;
          if ((st = time_run([&] { return run_family(FAM_MSD); }, &mb))) break;
          if (bbest == 0.0f || mb < bbest) {
            bbest = mb;
            bcap = cap;
          }
        }
        if (!st && bbest < tmsd[fl]) {
          h->fam_cap[FAM_MSD] = (int8_t)bcap;
        } else {
          h->use_box_msd = 0;
          h->fam_cap[FAM_MSD] = cap_msd[fl];
        }
      }
    }
  }
  if (st) {
    for (int f = 0; f < kFamilies; ++f) h->fam_cap[f] = -1;
    h->series_nt_flip = 0;
    h->use_box = 0;
    h->use_box_msd = 0;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

gpuqt_status gpuqt_schedule_rows(int32_t n_segments, const int64_t* seg_offsets, const int64_t* period,
                                 int32_t band_rows, int32_t pencil, int32_t cus, int32_t B, int32_t* block_of_row,
                                 int32_t* iter_of_row) {
  if (n_segments < 1 || !seg_offsets || !block_of_row || !iter_of_row || cus < 1 || !valid_B(B))
    return fail(GPUQT_ERR_ARG, "bad arguments to gpuqt_schedule_rows");
  if (band_rows < 0 || band_rows % 64) return fail(GPUQT_ERR_ARG, "band_rows must be a multiple of 64");
  std::vector<int64_t> off(seg_offsets, seg_offsets + n_segments + 1);
  if (off[0] != 0) return fail(GPUQT_ERR_ARG, "seg_offsets[0] must be 0");
  for (int s = 0; s < n_segments; ++s)
    if (off[s + 1] <= off[s]) return fail(GPUQT_ERR_ARG, "segments must be non-empty and ascending");
  const int64_t n = off[n_segments];
  if (n > INT32_MAX) return fail(GPUQT_ERR_ARG, "too many rows");
  std::vector<BlkPlan> plan;
  std::vector<int32_t> blk0, units;
  plan_blocks(off, cus, kPerCU, &plan, &blk0);
  bool banded = false;
  std::vector<int64_t> D(n_segments, 0);
  for (int s = 0; s < n_segments && period; ++s) {
    D[s] = period[s];
    banded = banded || (band_rows > 0 && D[s] > band_rows);
  }
  if (banded && pencil) {
    std::vector<int64_t> pw(n_segments, 0);
    banded = false;
    for (int s = 0; s < n_segments; ++s)
      if (D[s] >= 128) {
        pw[s] = band_rows;
        banded = true;
      }
    if (banded) pencil_units(off, D, pw, &units);
  } else if (banded) {
    banded_units(off, D, std::vector<int64_t>(n_segments, band_rows), &units);
  }
  const bool pen = banded && pencil;
  const int32_t* U = banded ? units.data() : nullptr;
  for (int64_t r = 0; r < n; ++r) block_of_row[r] = iter_of_row[r] = -1;
  const int RPI = kBlock / B;
  for (size_t lb = 0; lb < plan.size(); ++lb) {
    const BlkPlan& P = plan[lb];
    const int64_t total = pen ? pencil_seq_len(P) : row_seq_len(P, U);
    int32_t it = 0;
    for (int64_t pos0 = (int64_t)P.j * RPI; pos0 < total; pos0 += (int64_t)P.g * RPI, ++it) {
      for (int i = 0; i < RPI; ++i) {
        const int64_t pos = pos0 + i;
        if (pos >= total) break;
        const int64_t r = pen ? row_at_pencil(P, U, pos, B) : row_at(P, U, pos);
        if (r < 0) continue;
        if (r >= n || block_of_row[r] != -1) return fail(GPUQT_ERR_LAYOUT, "schedule visits a row twice");
        block_of_row[r] = (int32_t)lb;
        iter_of_row[r] = it;
      }
    }
  }
  return GPUQT_OK;
}

gpuqt_status gpuqt_set_variant(gpuqt_h hh, int32_t variant) {
  Handle* h = reinterpret_cast<Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  if (variant < 0 || ((variant >> 2) & 15) > kPerCU || ((variant >> 6) & 1 && !((variant >> 1) & 1)) ||
      (variant >> (8 + 3 * kFamilies + 2)))
    return fail(GPUQT_ERR_ARG,
                "variant must be bits 0-1 load variant, bits 2-5 a per-CU cap of 0..8, bit 6 the pencil "
                "order (with bit 1), bit 7 the series families' load flip, 3 bits per kernel family "
                "from bit 8, bit 26 the periodic-box Hermitian step and bit 27 the periodic-box MSD term");
  h->nt = variant & 1;
  h->banded = (variant >> 1) & 1;
  h->pencil = (variant >> 6) & 1;
  h->series_nt_flip = (variant >> 7) & 1;
  h->use_box = (variant >> (8 + 3 * kFamilies)) & 1;
  h->use_box_msd = (variant >> (8 + 3 * kFamilies + 1)) & 1;
  h->per_cu_cap = (variant >> 2) & 15;
  for (int f = 0; f < kFamilies; ++f) h->fam_cap[f] = (int8_t)(((variant >> (8 + 3 * f)) & 7) - 1);
  return GPUQT_OK;
}

gpuqt_status gpuqt_kpm_reconstruct(int32_t R, int32_t M, const double* C, int32_t n_E,
                                   const double* energies, double energy_max, double volume,
                                   int32_t jackson, double* out, void* stream) {
  if (R < 0 || M < 1 || n_E < 0 || n_E > 65536) return fail(GPUQT_ERR_ARG, "bad sizes");
  if (!(energy_max > 0) || !(volume > 0)) return fail(GPUQT_ERR_ARG, "energy_max and volume must be > 0");
  if (R == 0 || n_E == 0) return GPUQT_OK;
  if (!C || !energies || !out) return fail(GPUQT_ERR_ARG, "NULL pointer");
  const double pref = 2.0 / (M_PI * volume * energy_max);
  HIP_TRY(launch_kpm(R, M, C, n_E, energies, 1.0 / energy_max, pref, jackson ? 1 : 0, out,
                     static_cast<hipStream_t>(stream)));
  return GPUQT_OK;
}

gpuqt_status gpuqt_running_conductivity(int32_t mode, int32_t n_t, const double* dt, int32_t n_E,
                                        const double* y, double* sigma, void* stream) {
  if (mode != GPUQT_SIGMA_VAC && mode != GPUQT_SIGMA_MSD) return fail(GPUQT_ERR_ARG, "unknown mode");
  if (n_t < 0 || n_E < 0) return fail(GPUQT_ERR_ARG, "n_t and n_E must be >= 0");
  if (n_t == 0 || n_E == 0) return GPUQT_OK;
  if (!dt || !y || !sigma) return fail(GPUQT_ERR_ARG, "NULL pointer");
  if (overlap(sigma, y, (size_t)n_t * n_E * 8)) return fail(GPUQT_ERR_ARG, "sigma must not overlap y");
  HIP_TRY(launch_sigma(mode, n_t, dt, n_E, y, sigma, static_cast<hipStream_t>(stream)));
  return GPUQT_OK;
}

gpuqt_status gpuqt_transport_lengths(int32_t n_t, int32_t n_E, const double* rho, const double* vac0,
                                     const double* sigma, const double* msd, double* sigma_sc, double* v,
                                     double* tau, double* mfp, double* L, double* xi, void* stream) {
  if (n_t < 0 || n_E < 0) return fail(GPUQT_ERR_ARG, "n_t and n_E must be >= 0");
  if (n_E == 0) return GPUQT_OK;
  if (!rho) return fail(GPUQT_ERR_ARG, "rho is NULL");
  if ((sigma_sc && !sigma) || (v && !vac0) || ((tau || mfp) && !(sigma && vac0)) || ((L || xi) && !msd))
    return fail(GPUQT_ERR_ARG, "an output was asked for without the rows it is computed from");
  if ((sigma || msd || L) && n_t == 0) return fail(GPUQT_ERR_ARG, "rows given or asked for with n_t = 0");
  const size_t e8 = (size_t)n_E * 8, r8 = (size_t)n_t * n_E * 8;
  const void* ins[][2] = {{rho, (const void*)e8}, {vac0, (const void*)e8}, {sigma, (const void*)r8},
                          {msd, (const void*)r8}};
  const void* outs[][2] = {{sigma_sc, (const void*)e8}, {v, (const void*)e8}, {tau, (const void*)e8},
                           {mfp, (const void*)e8}, {L, (const void*)r8}, {xi, (const void*)e8}};
  for (auto& o : outs) {
    if (!o[0]) continue;
    const char* a = static_cast<const char*>(o[0]);
    for (auto& i : ins) {
      const char* b = static_cast<const char*>(i[0]);
      if (b && a < b + (size_t)i[1] && b < a + (size_t)o[1])
        return fail(GPUQT_ERR_ARG, "outputs must not overlap the inputs");
    }
  }
  TransportIO io{n_t, n_E, rho, vac0, sigma, msd, sigma_sc, v, tau, mfp, xi, L};
  HIP_TRY(launch_transport(io, static_cast<hipStream_t>(stream)));
  return GPUQT_OK;
}

gpuqt_status gpuqt_set_timing(gpuqt_h hh, int32_t enable) {
  Handle* h = reinterpret_cast<Handle*>(hh);
  if (!h) return fail(GPUQT_ERR_ARG, "NULL handle");
  h->timing = enable != 0;
  return GPUQT_OK;
}

gpuqt_status gpuqt_timing(gpuqt_h hh, double* ms, int64_t* launches) {
  Handle* h = reinterpret_cast<Handle*>(hh);
  if (!h || !ms || !launches) return fail(GPUQT_ERR_ARG, "NULL argument");
  for (int f = 0; f < GPUQT_K_COUNT; ++f) {
    ms[f] = 0.0;
    launches[f] = 0;
  }
  gpuqt_status st = GPUQT_OK;
  for (auto& r : h->timing_recs) {
    float t = 0.0f;
    if (st == GPUQT_OK) {
      hipError_t e = hipEventSynchronize(r.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
      if (e != hipSuccess) {
        st = fail(GPUQT_ERR_HIP, std::string("timing events: ") + hipGetErrorString(e));
      } else {
        ms[r.family] += t;
        launches[r.family] += r.launches;
      }
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  h->timing_recs.clear();
  return st;
}

gpuqt_status gpuqt_kpm_reconstruct_adjoint(int32_t R, int32_t M, const double* g, int32_t n_E,
                                           const double* energies, double energy_max, double volume,
                                           int32_t jackson, double* out, void* stream) {
  if (R < 0 || M < 1 || n_E < 0 || n_E > 65536) return fail(GPUQT_ERR_ARG, "bad sizes");
  if (!(energy_max > 0) || !(volume > 0)) return fail(GPUQT_ERR_ARG, "energy_max and volume must be > 0");
  if (R == 0) return GPUQT_OK;
  if (!g || !energies || !out) return fail(GPUQT_ERR_ARG, "NULL pointer");
  const double pref = 2.0 / (M_PI * volume * energy_max);
  HIP_TRY(launch_kpm_adjoint(R, M, g, n_E, energies, 1.0 / energy_max, pref, jackson ? 1 : 0, out,
                             static_cast<hipStream_t>(stream)));
  return GPUQT_OK;
}

gpuqt_status gpuqt_copy_probe(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst || (bytes & 15) || !aligned16(src) || !aligned16(dst))
    return fail(GPUQT_ERR_ARG, "copy probe needs 16-byte aligned buffers and a multiple of 16 bytes");
  if (overlap(src, dst, bytes)) return fail(GPUQT_ERR_ARG, "copy probe buffers overlap");
  HIP_TRY(launch_copy(static_cast<const double2*>(src), static_cast<double2*>(dst), bytes / 16,
                      static_cast<hipStream_t>(stream)));
  return GPUQT_OK;
}

}  // extern "C"
