// Readers for the input folder of the paper's program (Section 4.2): the model
// files neighbour.in, hopping.in, potential.in, position.in and the run files
// energy.in, time_step.in, para.in.  Host-only C++; the arrays they produce feed
// gpuqt_build_h through a gpuqt_h_desc.
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace gpuqt {
namespace {

struct Model {
  int64_t n = 0;
  int32_t max_nn = 0;
  std::vector<int32_t> nn, nbr;
  std::vector<double> hop;   // empty: every hopping is -1
  bool hop_complex = false;
  std::vector<double> onsite;
  std::vector<double> x;
  double length_x = 0.0, volume = 0.0;
  std::vector<double> energies, dt;
  int32_t n_r = 1, n_m = 1000, vac = 0, msd = 0;
  double energy_max = 10.0;
};

// Whole-file tokenizer with line tracking.
class Reader {
 public:
  bool open(const std::string& path) {
    path_ = path;
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::fseek(f, 0, SEEK_END);
    const long sz = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    buf_.resize(sz > 0 ? (size_t)sz + 1 : 1);
    const size_t got = sz > 0 ? std::fread(&buf_[0], 1, (size_t)sz, f) : 0;
    std::fclose(f);
    buf_[got] = '\0';
    p_ = buf_.c_str();
    line_ = 1;
    return true;
  }
  // next token on the current line (false at the end of the line or file)
  bool token(std::string* t) {
    while (*p_ == ' ' || *p_ == '\t' || *p_ == '\r') ++p_;
    if (*p_ == '\0' || *p_ == '\n') return false;
    const char* s = p_;
    while (*p_ && *p_ != ' ' && *p_ != '\t' && *p_ != '\r' && *p_ != '\n') ++p_;
    t->assign(s, p_ - s);
    return true;
  }
  bool next_line() {   // skip the rest of the line; false when no further line has content
    while (*p_ && *p_ != '\n') ++p_;
    if (*p_ == '\0') return false;
    ++p_;
    ++line_;
    return *p_ != '\0';
  }
  bool skip_blank_lines() {   // to the next non-blank line; false at the end of the file
    for (;;) {
      const char* q = p_;
      while (*q == ' ' || *q == '\t' || *q == '\r') ++q;
      if (*q == '\0') return false;
      if (*q != '\n') return true;
      p_ = q + 1;
      ++line_;
    }
  }
  bool get_int(int64_t* v) {
    std::string t;
    if (!token(&t)) return false;
    char* e = nullptr;
    errno = 0;
    const long long x = std::strtoll(t.c_str(), &e, 10);
    if (errno || *e) return false;
    *v = x;
    return true;
  }
  bool get_double(double* v) {
    std::string t;
    if (!token(&t)) return false;
    char* e = nullptr;
    errno = 0;
    const double x = std::strtod(t.c_str(), &e);
    if (errno == ERANGE || *e || !std::isfinite(x)) return false;
    *v = x;
    return true;
  }
  std::string where() const { return path_ + ":" + std::to_string(line_); }

 private:
  std::string buf_, path_;
  const char* p_ = nullptr;
  int64_t line_ = 1;
};

bool exists(const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  std::fclose(f);
  return true;
}

gpuqt_status bad(const Reader& r, const std::string& what) {
  return set_error(GPUQT_ERR_LAYOUT, r.where() + ": " + what);
}

gpuqt_status read_neighbour(const std::string& dir, Model* m) {
  Reader r;
  if (!r.open(dir + "/neighbour.in")) return set_error(GPUQT_ERR_ARG, "cannot open " + dir + "/neighbour.in");
  int64_t n = 0, k = 0;
  if (!r.get_int(&n) || !r.get_int(&k)) return bad(r, "expected the number of sites and the maximum neighbour count");
  if (n < 1 || n > INT32_MAX) return bad(r, "the number of sites must be in [1, 2^31)");
  if (k < 0 || k > 4096) return bad(r, "the maximum neighbour count must be in [0, 4096]");
  m->n = n;
  m->max_nn = (int32_t)k;
  m->nn.assign(n, 0);
  m->nbr.assign((size_t)n * (size_t)k, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (!r.next_line()) return bad(r, "expected " + std::to_string(n) + " site lines");
    int64_t c = 0;
    if (!r.get_int(&c) || c < 0 || c > k) return bad(r, "neighbour count of site " + std::to_string(i));
    m->nn[i] = (int32_t)c;
    for (int64_t s = 0; s < c; ++s) {
      int64_t j = 0;
      if (!r.get_int(&j) || j < 0 || j >= n) return bad(r, "neighbour index of site " + std::to_string(i));
      m->nbr[(size_t)i * k + s] = (int32_t)j;
    }
  }
  return GPUQT_OK;
}

gpuqt_status read_hopping(const std::string& dir, Model* m) {
  const std::string path = dir + "/hopping.in";
  if (!exists(path)) return GPUQT_OK;   // every hopping is -1
  Reader r;
  if (!r.open(path)) return set_error(GPUQT_ERR_ARG, "cannot open " + path);
  std::string kind;
  if (!r.token(&kind) || (kind != "real" && kind != "complex"))
    return bad(r, "the first line must be 'real' or 'complex'");
  m->hop_complex = kind == "complex";
  const int per = m->hop_complex ? 2 : 1;
  m->hop.assign((size_t)m->n * m->max_nn * per, 0.0);
  for (int64_t i = 0; i < m->n; ++i) {
    if (!r.next_line()) return bad(r, "expected " + std::to_string(m->n) + " site lines");
    for (int s = 0; s < m->nn[i] * per; ++s)
      if (!r.get_double(&m->hop[((size_t)i * m->max_nn) * per + s]))
        return bad(r, "hopping of site " + std::to_string(i));
  }
  return GPUQT_OK;
}

gpuqt_status read_column(const std::string& path, int64_t count, std::vector<double>* v) {
  Reader r;
  if (!r.open(path)) return set_error(GPUQT_ERR_ARG, "cannot open " + path);
  v->assign(count, 0.0);
  for (int64_t i = 0; i < count; ++i) {
    if (i > 0 && !r.next_line()) return bad(r, "expected " + std::to_string(count) + " lines");
    if (!r.get_double(&(*v)[i])) return bad(r, "value " + std::to_string(i));
  }
  return GPUQT_OK;
}

gpuqt_status read_counted(const std::string& path, std::vector<double>* v) {
  Reader r;
  if (!r.open(path)) return set_error(GPUQT_ERR_ARG, "cannot open " + path);
  int64_t c = 0;
  if (!r.get_int(&c) || c < 0 || c > (int64_t)1 << 24) return bad(r, "expected the number of values");
  v->assign(c, 0.0);
  for (int64_t i = 0; i < c; ++i) {
    if (!r.next_line()) return bad(r, "expected " + std::to_string(c) + " values");
    if (!r.get_double(&(*v)[i])) return bad(r, "value " + std::to_string(i));
  }
  return GPUQT_OK;
}

gpuqt_status read_para(const std::string& dir, Model* m) {
  const std::string path = dir + "/para.in";
  if (!exists(path)) return GPUQT_OK;
  Reader r;
  if (!r.open(path)) return set_error(GPUQT_ERR_ARG, "cannot open " + path);
  for (;;) {
    if (!r.skip_blank_lines()) break;
    std::string key;
    r.token(&key);
    if (key == "calculate_vac") {
      m->vac = 1;
    } else if (key == "calculate_msd") {
      m->msd = 1;
    } else if (key == "number_of_random_vectors") {
      int64_t v = 0;
      if (!r.get_int(&v) || v < 1 || v > 1000000) return bad(r, "number_of_random_vectors needs a count >= 1");
      m->n_r = (int32_t)v;
    } else if (key == "number_of_moments") {
      int64_t v = 0;
      if (!r.get_int(&v) || v < 1 || v > 10000000) return bad(r, "number_of_moments needs a count >= 1");
      m->n_m = (int32_t)v;
    } else if (key == "energy_max") {
      double v = 0.0;
      if (!r.get_double(&v) || !(v > 0)) return bad(r, "energy_max needs a positive value");
      m->energy_max = v;
    } else {
      return bad(r, "unknown keyword '" + key + "'");
    }
    std::string extra;
    if (r.token(&extra)) return bad(r, "unexpected '" + extra + "' after " + key);
    if (!r.next_line()) break;
  }
  return GPUQT_OK;
}

}  // namespace
}  // namespace gpuqt

using namespace gpuqt;

struct gpuqt_model_s : Model {};

extern "C" {

gpuqt_status gpuqt_model_load(const char* dir, gpuqt_model* out) {
  if (!dir || !out) return set_error(GPUQT_ERR_ARG, "NULL argument");
  *out = nullptr;
  const std::string d(dir);
  gpuqt_model_s* m = new gpuqt_model_s();
  gpuqt_status st;
  if ((st = read_neighbour(d, m)) || (st = read_hopping(d, m))) {
    delete m;
    return st;
  }
  if (exists(d + "/potential.in") && (st = read_column(d + "/potential.in", m->n, &m->onsite))) {
    delete m;
    return st;
  }
  {
    Reader r;
    if (!r.open(d + "/position.in")) {
      delete m;
      return set_error(GPUQT_ERR_ARG, "cannot open " + d + "/position.in");
    }
    if (!r.get_double(&m->length_x) || !r.get_double(&m->volume) || !(m->volume > 0)) {
      st = bad(r, "expected the length along x and a positive volume");
      delete m;
      return st;
    }
    m->x.assign(m->n, 0.0);
    for (int64_t i = 0; i < m->n; ++i) {
      if (!r.next_line() || !r.get_double(&m->x[i])) {
        st = bad(r, "position of site " + std::to_string(i));
        delete m;
        return st;
      }
    }
  }
  if ((st = read_counted(d + "/energy.in", &m->energies)) || (st = read_para(d, m))) {
    delete m;
    return st;
  }
  if ((m->vac || m->msd) && (st = read_counted(d + "/time_step.in", &m->dt))) {
    delete m;
    return st;
  }
  *out = m;
  return GPUQT_OK;
}

gpuqt_status gpuqt_model_desc(gpuqt_model m, gpuqt_h_desc* d) {
  if (!m || !d) return set_error(GPUQT_ERR_ARG, "NULL argument");
  std::memset(d, 0, sizeof(*d));
  d->n = m->n;
  d->max_nn = m->max_nn;
  d->nn = m->nn.data();
  d->nbr = m->nbr.data();
  d->hop = m->hop.empty() ? nullptr : m->hop.data();
  d->hop_is_complex = m->hop_complex ? 1 : 0;
  d->n_class = 1;
  d->onsite = m->onsite.empty() ? nullptr : m->onsite.data();
  d->x = m->x.data();
  d->length_x = m->length_x;
  d->volume = m->volume;
  d->energy_max = m->energy_max;
  return GPUQT_OK;
}

gpuqt_status gpuqt_model_params(gpuqt_model m, gpuqt_model_params_t* p) {
  if (!m || !p) return set_error(GPUQT_ERR_ARG, "NULL argument");
  p->n_random_vectors = m->n_r;
  p->n_moments = m->n_m;
  p->energy_max = m->energy_max;
  p->calculate_vac = m->vac;
  p->calculate_msd = m->msd;
  p->n_energies = (int32_t)m->energies.size();
  p->energies = m->energies.data();
  p->n_time_steps = (int32_t)m->dt.size();
  p->time_steps = m->dt.empty() ? nullptr : m->dt.data();
  return GPUQT_OK;
}

void gpuqt_model_free(gpuqt_model m) { delete m; }

}  // extern "C"
