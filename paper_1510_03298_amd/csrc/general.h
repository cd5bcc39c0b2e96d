// general.h -- the generic-GEMM solver of the lambda path (general.cpp): models of c >= 1 tensor
// components (Sec. 2, eq. fivenew), and single-component models beyond the slab kernels' limits.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "glam.h"

namespace glam {

struct GenComponent {
  int64_t p[3];          // p_{r,1..3}
  const double* X[3];    // device FP64 factors, X[j] n_j x p_{r,j} column-major
};

struct GenProblem {
  int64_t n[3];                      // d = 3 (a d = 2 model is lifted with a 1 x 1 middle factor)
  std::vector<GenComponent> comps;   // theta = (vec(Theta_1), ..., vec(Theta_c))
  const double* Y;
  const double* obs_w;
  int family;
  const double* pen_w;               // length sum_r p_r, or NULL
};

// Fits the lambda path; on error *why holds the reason.  The options and result arrays are
// validated by the caller (check_fit_options).
int general_fit_path(const GenProblem& prob, const glam_options* opt, glam_result* res, std::string* why);

// The checks of glam_fit_path on options and result arrays (fit.cpp).
int check_fit_options(const glam_options* opt, const glam_result* res, int family, bool has_obs_w, std::string* why);

}  // namespace glam
