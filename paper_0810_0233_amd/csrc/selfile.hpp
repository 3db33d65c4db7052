// selfile.hpp -- selector weights files, host code only (no HIP): the library
// builds it with the kernels, and the CPU tests build it alone under the
// address and undefined-behaviour sanitizers.
#pragma once
#include <string>

#include "../../include/ccfmm.h"

namespace ccfmm {
// the selector's candidates: orders kSelPLo..kSelPHi, angles kSelTheta
// (network output (p - kSelPLo) * 5 + angle index)
inline constexpr unsigned kSelPLo = 2, kSelPHi = 6;
inline constexpr double kSelTheta[5] = {0.3, 0.4, 0.5, 0.6, 0.7};

// Write h_params [CCFMM_MLP_PARAMS] to path.  CCFMM_OK, or CCFMM_EINVAL with
// *err set.
int selfile_write(const char* path, const float* h_params, std::string* err);
// Read path into h_params.  CCFMM_OK; CCFMM_W_NOWEIGHTS if the file does not
// exist (h_params untouched); CCFMM_EINVAL with *err set for any other problem
// (h_params untouched).
int selfile_read(const char* path, float* h_params, std::string* err);
}  // namespace ccfmm
