// Tuning choices that are not made inside one handle: a process-wide cache of
// kernel variants keyed by the configuration they were measured on, the
// vector-block width for a number of random vectors, and the sliced-ELL slice
// height (Section 4.2.7 notes that the random vectors are independent, so
// their grouping into blocks is free to choose).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "internal.h"

using namespace gpuqt;

namespace {

std::mutex g_mu;
std::map<std::string, int32_t> g_cache;

// Everything the variant choice depends on: the device architecture, the
// problem size (log2 bucket), the row structure (fixed width or widest
// slice, slice height), the hopping storage, the segment count, the row
// period bucket and which block widths have a banded order, and B.
gpuqt_status tune_key(const Handle* h, int B, std::string* key) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, h->device) != hipSuccess)
    return set_error(GPUQT_ERR_HIP, "hipGetDeviceProperties failed");
  std::string arch = prop.gcnArchName;
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch.resize(c);
  int64_t period = 0;
  for (int64_t D : h->seg_period) period = std::max(period, D);
  int mask = 0;
  for (int b = 0; b < kNumB; ++b)
    if (h->d_units[b]) mask |= 1 << b;
  std::ostringstream o;
  o << arch << " n" << (int)std::floor(std::log2((double)std::max<int64_t>(h->n, 1))) << " K" << h->uniform_width
    << " w" << h->max_width << " S" << h->S << " h" << h->hop_mode << " s" << h->n_seg << " p"
    << (period > 0 ? (int)std::floor(std::log2((double)period)) : -1) << " m" << mask << " B" << B;
  *key = o.str();
  return GPUQT_OK;
}

bool valid_B(int B) { return B == 1 || B == 2 || B == 4 || B == 8 || B == 16; }

}  // namespace

gpuqt_status gpuqt_tune_cache_key(gpuqt_h hh, int32_t B, char* buf, size_t len) {
  const Handle* h = reinterpret_cast<const Handle*>(hh);
  if (!h || !buf || len == 0 || !valid_B(B)) return set_error(GPUQT_ERR_ARG, "bad arguments to gpuqt_tune_cache_key");
  std::string key;
  gpuqt_status st = tune_key(h, B, &key);
  if (st) return st;
  if (key.size() + 1 > len) return set_error(GPUQT_ERR_ARG, "key buffer too small");
  std::memcpy(buf, key.c_str(), key.size() + 1);
  return GPUQT_OK;
}

gpuqt_status gpuqt_tune_cache_load(const char* path) {
  if (!path) return set_error(GPUQT_ERR_ARG, "path is NULL");
  std::ifstream f(path);
  if (!f) return set_error(GPUQT_ERR_ARG, std::string("cannot open ") + path);
  std::map<std::string, int32_t> add;
  std::string line;
  int ln = 0;
  while (std::getline(f, line)) {
    ++ln;
    if (line.empty() || line[0] == '#') continue;
    const size_t t = line.rfind('\t');
    char* end = nullptr;
    const long v = t == std::string::npos ? -1 : std::strtol(line.c_str() + t + 1, &end, 10);
    if (t == std::string::npos || t == 0 || v < 0 || v > INT32_MAX || (end && *end != '\0'))
      return set_error(GPUQT_ERR_LAYOUT, std::string(path) + ":" + std::to_string(ln) +
                                             ": expected <key>TAB<variant code>");
    add[line.substr(0, t)] = (int32_t)v;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : add) g_cache[kv.first] = kv.second;
  return GPUQT_OK;
}

gpuqt_status gpuqt_tune_cache_save(const char* path) {
  if (!path) return set_error(GPUQT_ERR_ARG, "path is NULL");
  std::map<std::string, int32_t> snap;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    snap = g_cache;
  }
  std::ofstream f(path);
  if (!f) return set_error(GPUQT_ERR_ARG, std::string("cannot write ") + path);
  f << "# kernel variant codes chosen by gpuqt_autotune: <configuration key>\\t<code>\n";
  for (auto& kv : snap) f << kv.first << '\t' << kv.second << '\n';
  return f ? GPUQT_OK : set_error(GPUQT_ERR_ARG, std::string("write failed: ") + path);
}

void gpuqt_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
}

gpuqt_status gpuqt_autotune_cached(gpuqt_h hh, int32_t B, void* ws, size_t ws_bytes, void* stream,
                                   double* times_us, int32_t* from_cache) {
  Handle* h = reinterpret_cast<Handle*>(hh);
  if (!h) return set_error(GPUQT_ERR_ARG, "NULL handle");
  if (!valid_B(B)) return set_error(GPUQT_ERR_UNSUPPORTED, "B must be 1, 2, 4, 8 or 16");
  std::string key;
  gpuqt_status st = tune_key(h, B, &key);
  if (st) return st;
  int32_t code = -1;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) code = it->second;
  }
  if (code >= 0 && gpuqt_set_variant(hh, code) == GPUQT_OK) {
    if (times_us)
      for (int v = 0; v < kTuneTimes; ++v) times_us[v] = 0.0;
    if (from_cache) *from_cache = 1;
    return GPUQT_OK;
  }
  if ((st = gpuqt_autotune(hh, B, ws, ws_bytes, stream, times_us))) return st;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = h->variant_code();
  }
  if (from_cache) *from_cache = 0;
  return GPUQT_OK;
}

gpuqt_status gpuqt_autotune_block(gpuqt_h hh, int32_t n_vectors, void* ws, size_t ws_bytes, void* stream,
                                  int32_t* best_B, double* us_per_vector_step) {
  Handle* h = reinterpret_cast<Handle*>(hh);
  if (!h || !best_B || n_vectors < 1) return set_error(GPUQT_ERR_ARG, "bad arguments to gpuqt_autotune_block");
  if (us_per_vector_step)
    for (int i = 0; i < kNumB; ++i) us_per_vector_step[i] = 0.0;
  double best = 0.0;
  int bestB = 1;
  for (int lb = 0; lb < kNumB; ++lb) {
    const int B = 1 << lb;
    if (B > n_vectors) break;
    size_t need = 0;
    gpuqt_status st = gpuqt_workspace_size(hh, GPUQT_OP_AUTOTUNE, B, 0, 0, &need);
    if (st) return st;
    if (ws_bytes < need) break;   // the workspace bounds the widest block tried
    double t[kTuneTimes] = {};
    if ((st = gpuqt_autotune(hh, B, ws, ws_bytes, stream, t))) return st;
    double us = 0.0;
    for (double x : t)
      if (x > 0.0 && (us == 0.0 || x < us)) us = x;
    const double per = us / B;   // one Hermitian moment step of the block, per vector
    if (us_per_vector_step) us_per_vector_step[lb] = per;
    if (per > 0.0 && (best == 0.0 || per < best)) {
      best = per;
      bestB = B;
    }
    std::string key;
    if ((st = tune_key(h, B, &key))) return st;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = h->variant_code();
  }
  if (best == 0.0) return set_error(GPUQT_ERR_WORKSPACE, "workspace too small for a block of one vector");
  *best_B = bestB;
  // leave the handle tuned for the chosen width (its cached variant)
  std::string key;
  gpuqt_status st = tune_key(h, bestB, &key);
  if (st) return st;
  int32_t code = -1;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    code = g_cache[key];
  }
  return gpuqt_set_variant(hh, code);
}

gpuqt_status gpuqt_build_h_tuned(const gpuqt_h_desc* desc, int32_t B, void* stream, gpuqt_h* out,
                                 int32_t* slice_height, double* us_per_step) {
  if (!desc || !out || !valid_B(B)) return set_error(GPUQT_ERR_ARG, "bad arguments to gpuqt_build_h_tuned");
  *out = nullptr;
  static const int kHeights[4] = {32, 64, 128, 256};
  if (us_per_step)
    for (int i = 0; i < 4; ++i) us_per_step[i] = 0.0;
  gpuqt_h best = nullptr;
  double best_us = 0.0;
  int best_S = 0;
  for (int i = 0; i < 4; ++i) {
    gpuqt_h_desc d = *desc;
    d.slice_height = kHeights[i];
    gpuqt_h h = nullptr;
    gpuqt_status st = gpuqt_build_h(&d, stream, &h);
    if (st) {
      if (best) gpuqt_destroy_h(best);
      return st;
    }
    size_t need = 0;
    void* ws = nullptr;
    double t[kTuneTimes] = {};
    if ((st = gpuqt_workspace_size(h, GPUQT_OP_AUTOTUNE, B, 0, 0, &need)) == GPUQT_OK) {
      if (hipMalloc(&ws, need) != hipSuccess) {
        ws = nullptr;
        st = set_error(GPUQT_ERR_NOMEM, "workspace allocation failed while tuning the slice height");
      } else {
        st = gpuqt_autotune(h, B, ws, need, stream, t);
        (void)hipFree(ws);
      }
    }
    if (st) {
      gpuqt_destroy_h(h);
      if (best) gpuqt_destroy_h(best);
      return st;
    }
    double us = 0.0;
    for (double x : t)
      if (x > 0.0 && (us == 0.0 || x < us)) us = x;
    if (us_per_step) us_per_step[i] = us;
    if (!best || (us > 0.0 && us < best_us)) {
      if (best) gpuqt_destroy_h(best);
      best = h;
      best_us = us;
      best_S = kHeights[i];
    } else {
      gpuqt_destroy_h(h);
    }
  }
  *out = best;
  if (slice_height) *slice_height = best_S;
  return GPUQT_OK;
}
