// Exercises the selector weights-file writer and reader (host code of the
// library, selfile.cpp) under the address and undefined-behaviour sanitizers:
// a round trip, a missing file, and refusals of truncated, extended, altered,
// foreign and unreadable files.  Exit status 0 when every call returned what
// it should.  Usage: selfile_driver <scratch directory>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_0810_0233_amd/csrc/selfile.hpp"

static int g_bad = 0;
#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      g_bad++;                                                         \
    }                                                                  \
  } while (0)

static std::vector<unsigned char> slurp(const std::string& p) {
  std::vector<unsigned char> b;
  FILE* f = std::fopen(p.c_str(), "rb");
  if (!f) return b;
  int c;
  while ((c = std::fgetc(f)) != EOF) b.push_back((unsigned char)c);
  std::fclose(f);
  return b;
}

static void spit(const std::string& p, const std::vector<unsigned char>& b) {
  FILE* f = std::fopen(p.c_str(), "wb");
  if (!f) return;
  if (!b.empty()) std::fwrite(b.data(), 1, b.size(), f);
  std::fclose(f);
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const std::string dir = argv[1];
  std::vector<float> P(CCFMM_MLP_PARAMS), R(CCFMM_MLP_PARAMS, 7.f);
  for (int i = 0; i < CCFMM_MLP_PARAMS; i++) P[i] = 0.001f * (float)(i % 977) - 0.3f;
  std::string err;
  const std::string good = dir + "/good.ccsel";
  CHECK(ccfmm::selfile_write(good.c_str(), P.data(), &err) == CCFMM_OK);
  CHECK(ccfmm::selfile_read(good.c_str(), R.data(), &err) == CCFMM_OK);
  CHECK(std::memcmp(P.data(), R.data(), sizeof(float) * P.size()) == 0);
  CHECK(ccfmm::selfile_read((dir + "/absent.ccsel").c_str(), R.data(), &err) == CCFMM_W_NOWEIGHTS);
  CHECK(ccfmm::selfile_read(nullptr, R.data(), &err) == CCFMM_EINVAL);
  CHECK(ccfmm::selfile_write(nullptr, P.data(), &err) == CCFMM_EINVAL);
  CHECK(ccfmm::selfile_read(dir.c_str(), R.data(), &err) == CCFMM_EINVAL);  // a directory
  const std::vector<unsigned char> b = slurp(good);
  CHECK(!b.empty());
  const std::string bad = dir + "/bad.ccsel";
  // truncated at every header field boundary and inside the parameters
  const size_t cuts[] = {0, 1, 7, 8, 12, 35, 36, 75, 76, 77, 1000, b.size() - 9, b.size() - 8, b.size() - 1};
  for (size_t cut : cuts) {
    spit(bad, std::vector<unsigned char>(b.begin(), b.begin() + (long)cut));
    CHECK(ccfmm::selfile_read(bad.c_str(), R.data(), &err) == CCFMM_EINVAL);
  }
  // one byte more
  std::vector<unsigned char> longer = b;
  longer.push_back(0);
  spit(bad, longer);
  CHECK(ccfmm::selfile_read(bad.c_str(), R.data(), &err) == CCFMM_EINVAL);
  // one bit flipped anywhere: header, angles, parameters, hash
  for (size_t at = 0; at < b.size(); at += 97) {
    std::vector<unsigned char> f = b;
    f[at] ^= 0x10;
    spit(bad, f);
    CHECK(ccfmm::selfile_read(bad.c_str(), R.data(), &err) == CCFMM_EINVAL);
  }
  // garbage of the right length
  std::vector<unsigned char> g(b.size());
  unsigned s = 12345;
  for (auto& c : g) c = (unsigned char)((s = s * 1103515245u + 12345u) >> 16);
  spit(bad, g);
  CHECK(ccfmm::selfile_read(bad.c_str(), R.data(), &err) == CCFMM_EINVAL);
  // a refused read leaves the output untouched
  std::vector<float> keep(CCFMM_MLP_PARAMS, 3.f), out = keep;
  CHECK(ccfmm::selfile_read(bad.c_str(), out.data(), &err) == CCFMM_EINVAL);
  CHECK(out == keep);
  if (g_bad) return 1;
  std::printf("selector file driver OK\n");
  return 0;
}
