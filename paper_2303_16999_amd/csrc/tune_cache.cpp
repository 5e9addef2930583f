// The autotuner's table on disk: a small JSON file, written and read only by
// this library.
//
//   {"format": "spmm-autotune-2", "device": "<arch>/<CUs>", "hip_runtime": N,
//    "entries": [{"b": 16, "w": 1, "x": 1, "y": 1, "density_class": 4,
//                 "n_class": 12, "dense": 0, "variant": 264}, ...]}
//
// An entry maps a plan class (block size, dtypes as spmm_dtype_t codes,
// density class = round(-log2 d), n class = exponent of the power of two at
// or above n, whether the plan keeps a dense copy) to the variant code the
// tuner chose. A file written for another
// device or HIP runtime is ignored, as is one this reader cannot parse: the
// tuner then measures again and overwrites it.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <unistd.h>

#include "internal.h"

namespace spmm {
namespace {

constexpr const char* kFormat = "spmm-autotune-2";

bool device_identity(std::string* device, int* runtime) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  int rt = 0;
  if (hipRuntimeGetVersion(&rt) != hipSuccess) return false;
  *device = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
  *runtime = rt;
  return true;
}

// The string value of "key" in text (no escapes: the writer emits none).
bool find_string(const std::string& text, const char* key, std::string* out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = text.find(k);
  if (p == std::string::npos) return false;
  p = text.find(':', p + k.size());
  if (p == std::string::npos) return false;
  p = text.find('"', p);
  if (p == std::string::npos) return false;
  const size_t q = text.find('"', p + 1);
  if (q == std::string::npos) return false;
  *out = text.substr(p + 1, q - p - 1);
  return true;
}

// The integer value of "key" in text[lo, hi).
bool find_int(const std::string& text, size_t lo, size_t hi, const char* key, long long* out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = text.find(k, lo);
  if (p == std::string::npos || p >= hi) return false;
  p = text.find(':', p + k.size());
  if (p == std::string::npos || p >= hi) return false;
  const char* s = text.c_str() + p + 1;
  char* end = nullptr;
  const long long v = strtoll(s, &end, 10);
  if (end == s || (size_t)(end - text.c_str()) > hi) return false;
  *out = v;
  return true;
}

}  // namespace

bool tune_cache_load(const char* path, std::map<TuneKey, int32_t>& table) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  std::string fmt, device, my_device;
  long long runtime = 0;
  int my_runtime = 0;
  if (!find_string(text, "format", &fmt) || fmt != kFormat) return false;
  if (!find_string(text, "device", &device) || !find_int(text, 0, text.size(), "hip_runtime", &runtime)) return false;
  if (!device_identity(&my_device, &my_runtime) || device != my_device || runtime != my_runtime) return false;
  size_t p = text.find("\"entries\"");
  if (p == std::string::npos) return false;
  std::map<TuneKey, int32_t> got;
  while ((p = text.find('{', p + 1)) != std::string::npos) {
    const size_t q = text.find('}', p);
    if (q == std::string::npos) return false;
    long long v[8];
    const char* keys[8] = {"b", "w", "x", "y", "density_class", "n_class", "dense", "variant"};
    for (int i = 0; i < 8; ++i)
      if (!find_int(text, p, q, keys[i], &v[i])) return false;
    if (!valid_variant((int32_t)v[0], (int32_t)v[7]) || v[7] == 0 || (v[6] != 0 && v[6] != 1)) return false;
    if (v[6] == 0 && (v[7] >> kFormShift) == 3) return false;  // the dense form needs a dense copy
    if ((v[7] >> kFormShift) == 5) return false;                // the one-launch form is for dynamic calls
    got[TuneKey((int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5], (int)v[6])] = (int32_t)v[7];
    p = q;
  }
  for (const auto& kv : got) table.emplace(kv.first, kv.second);  // entries measured here win
  return true;
}

bool tune_cache_save(const char* path, const std::map<TuneKey, int32_t>& table) {
  std::string device;
  int runtime = 0;
  if (!device_identity(&device, &runtime)) return false;
  std::ostringstream o;
  o << "{\"format\": \"" << kFormat << "\", \"device\": \"" << device << "\", \"hip_runtime\": " << runtime
    << ",\n \"entries\": [";
  bool first = true;
  for (const auto& kv : table) {
    const TuneKey& k = kv.first;
    o << (first ? "\n  " : ",\n  ") << "{\"b\": " << std::get<0>(k) << ", \"w\": " << std::get<1>(k)
      << ", \"x\": " << std::get<2>(k) << ", \"y\": " << std::get<3>(k) << ", \"density_class\": " << std::get<4>(k)
      << ", \"n_class\": " << std::get<5>(k) << ", \"dense\": " << std::get<6>(k)
      << ", \"variant\": " << kv.second << "}";
    first = false;
  }
  o << "\n]}\n";
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
    if (!f) return false;
    f << o.str();
    if (!f.good()) return false;
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace spmm
