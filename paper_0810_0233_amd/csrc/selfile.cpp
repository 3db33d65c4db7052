// selfile.cpp -- selector weights files: writing, and reading with every
// field checked (the file may come from anywhere).  Host code only.
//
// Layout (little-endian): "CCFMMSEL", uint32 version, inputs, hidden width,
// outputs, parameter count, lowest and highest candidate order, FP64
// candidate angles [5], FP32 parameters, uint64 FNV-1a hash of all preceding
// bytes.
#include "selfile.hpp"

#include <cerrno>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

namespace ccfmm {

static int set_err(std::string* err, const std::string& msg) {
  if (err) *err = msg;
  return CCFMM_EINVAL;
}
static const char kSelMagic[8] = {'C', 'C', 'F', 'M', 'M', 'S', 'E', 'L'};
constexpr uint32_t kSelVersion = 1;
constexpr size_t kSelHeaderBytes = 8 + 7 * 4 + 5 * 8;
constexpr size_t kSelFileBytes = kSelHeaderBytes + 4 * (size_t)CCFMM_MLP_PARAMS + 8;

// FNV-1a, 64-bit
static uint64_t fnv1a64(const unsigned char* p, size_t n) {
  uint64_t h = 14695981039346656037ull;
  for (size_t i = 0; i < n; i++) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

template <typename V>
static void put(std::vector<unsigned char>& b, V v) {
  unsigned char t[sizeof(V)];
  std::memcpy(t, &v, sizeof(V));
  b.insert(b.end(), t, t + sizeof(V));
}
template <typename V>
static V get(const unsigned char* p) {
  V v;
  std::memcpy(&v, p, sizeof(V));
  return v;
}

int selfile_write(const char* path, const float* h_params, std::string* err) {
  if (!path || !h_params) return set_err(err, "selector weights: NULL path or parameters");
  std::vector<unsigned char> b;
  b.reserve(kSelFileBytes);
  b.insert(b.end(), kSelMagic, kSelMagic + 8);
  put<uint32_t>(b, kSelVersion);
  put<uint32_t>(b, CCFMM_MLP_IN);
  put<uint32_t>(b, CCFMM_MLP_HIDDEN);
  put<uint32_t>(b, CCFMM_MLP_OUT);
  put<uint32_t>(b, CCFMM_MLP_PARAMS);
  put<uint32_t>(b, (uint32_t)kSelPLo);
  put<uint32_t>(b, (uint32_t)kSelPHi);
  for (double t : kSelTheta) put<double>(b, t);
  for (int i = 0; i < CCFMM_MLP_PARAMS; i++) put<float>(b, h_params[i]);
  put<uint64_t>(b, fnv1a64(b.data(), b.size()));
  FILE* f = std::fopen(path, "wb");
  if (!f) return set_err(err, std::string("selector weights: cannot create ") + path);
  const size_t w = std::fwrite(b.data(), 1, b.size(), f);
  const int c = std::fclose(f);
  if (w != b.size() || c != 0) return set_err(err, std::string("selector weights: cannot write ") + path);
  return CCFMM_OK;
}

int selfile_read(const char* path, float* h_params, std::string* err) {
  if (!path || !h_params) return set_err(err, "selector weights: NULL path or parameters");
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    if (errno == ENOENT) {
      if (err) *err = std::string("selector weights file not found: ") + path;
      return CCFMM_W_NOWEIGHTS;
    }
    return set_err(err, std::string("selector weights: cannot open ") + path);
  }
  std::vector<unsigned char> b(kSelFileBytes + 1);
  const size_t r = std::fread(b.data(), 1, b.size(), f);
  std::fclose(f);
  const std::string what = std::string("selector weights ") + path + ": ";
  if (r != kSelFileBytes) return set_err(err, what + "wrong size (truncated or not a weights file)");
  if (std::memcmp(b.data(), kSelMagic, 8) != 0) return set_err(err, what + "not a weights file");
  const unsigned char* p = b.data() + 8;
  if (get<uint32_t>(p) != kSelVersion) return set_err(err, what + "unknown version");
  if (get<uint32_t>(p + 4) != CCFMM_MLP_IN || get<uint32_t>(p + 8) != CCFMM_MLP_HIDDEN ||
      get<uint32_t>(p + 12) != CCFMM_MLP_OUT || get<uint32_t>(p + 16) != CCFMM_MLP_PARAMS)
    return set_err(err, what + "network shape differs from this library's");
  if (get<uint32_t>(p + 20) != kSelPLo || get<uint32_t>(p + 24) != kSelPHi)
    return set_err(err, what + "candidate orders differ from this library's");
  for (int t = 0; t < 5; t++)
    if (get<double>(p + 28 + 8 * t) != kSelTheta[t]) return set_err(err, what + "candidate angles differ");
  const size_t body = kSelFileBytes - 8;
  if (get<uint64_t>(b.data() + body) != fnv1a64(b.data(), body)) return set_err(err, what + "checksum mismatch");
  for (int i = 0; i < CCFMM_MLP_PARAMS; i++) h_params[i] = get<float>(b.data() + kSelHeaderBytes + 4 * (size_t)i);
  return CCFMM_OK;
}

}  // namespace ccfmm
