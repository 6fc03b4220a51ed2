// Host-side helpers of the single-grid driver (api.hip) used by the ensemble
// driver (ensemble.hip).
#pragma once

#include <vector>

#include "../../include/biofilm.h"
#include "kernels.hpp"

namespace bf {

constexpr int kCoarseN = 4;                                  // coarsest grid: 5 x 4 nodes
constexpr int kCoarseSize = (kCoarseN + 1) * kCoarseN;

int host_fail(int code, const char* msg);                    // sets bf_last_error
OpDesc host_level_op(int op, int n, double c);               // operator of one level
// Smoothing polynomial of a level (a[k], g[k] of the three-term recurrence); returns the degree.
int host_smoother(int op, int n, double c, const bf_solver_opts& o, double* a, double* g);
// Exact solution operator of the 5 x 4 grid (20 x 20, row-major).
int host_coarse_operator(int op, double c, std::vector<double>& G);
double host_column_sq(const OpDesc& A);                      // sum_j A_jk^2, interior column
void host_default_opts(int op, bf_solver_opts* o);
int host_check_opts(const bf_solver_opts& o);

}  // namespace bf
