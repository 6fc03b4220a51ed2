// Host side of the C ABI: grid and multigrid hierarchy, V-cycle orchestration,
// Krylov drivers (CG and GMRES in the weighted inner product), and the time
// step.  Every arithmetic step on fields runs in the kernels of kernels.hip;
// the host only sequences launches and reads convergence scalars.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/biofilm.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace bf;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(BF_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                              \
  } while (0)

#define TRY(expr)            \
  do {                       \
    int s_ = (expr);         \
    if (s_ < 0) return s_;   \
  } while (0)

// One multigrid level's fields, stored in T (float64, or float32 for the
// mixed-precision V-cycle).
template <typename T>
struct LevelT {
  int n = 0;
  int64_t npts = 0;
  T* xa = nullptr;  // iterate buffers (ping-pong)
  T* xb = nullptr;
  T* r = nullptr;   // residual
  T* b = nullptr;   // right-hand side (levels >= 1)
  T* m = nullptr;   // node mobilities of the variable-mobility V-cycle (on first use)
};
using Level = LevelT<double>;

constexpr int kCoarseN = 4;
constexpr int kCoarseSize = (kCoarseN + 1) * kCoarseN;

// Internal operator code of the variable-mobility Cahn-Hilliard operator
// I + c L_m L (bf_solve_ch_mob): applied by its own double-double kernel,
// solved by GMRES, preconditioned by the constant-mobility V-cycle.
constexpr int kOpMob = 3;

}  // namespace

struct bf_grid {
  int n = 0;
  int64_t npts = 0;
  hipStream_t stream = nullptr;
  std::vector<Level> lv;
  std::vector<LevelT<float>> lvf;  // float32 hierarchy (allocated on first mixed use)
  float* r32 = nullptr;            // float32 copy of the V-cycle's level-0 input
  float* z32 = nullptr;            // float32 V-cycle output read by the mixed CG step
  bool want_z32 = false;           // the float32 V-cycle writes z32 instead of z
  double *r = nullptr, *z = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr;
  double *work_b = nullptr;   // Cahn-Hilliard right-hand side inside bf_step
  double *work_p = nullptr;   // projected pressure right-hand side
  double *work_e = nullptr;   // adjoint: W^{-1} eta (allocated on first use)
  double *work_mu = nullptr;  // chemical potential of the right-hand side
  double *work_m = nullptr;   // mobility field of bf_step_ch_mob (allocated on first use)
  const double* mob = nullptr;  // mobility field of the current variable-mobility solve
  double mob_pre = 0.0;         // the mean rounded to 6 bits (preconditioner coefficient)
  double* scal = nullptr;     // device scalars (kNumSlots)
  double* partials = nullptr; // reduction partials (kMaxRedBlocks * 72)
  double* coarse_ch = nullptr;
  double* coarse_lap = nullptr;
  double* coarse_helm = nullptr;
  double cached_c = -1.0;
  double cached_beta = -1.0;
  int32_t* counter = nullptr;
  double* h_scal = nullptr;   // pinned host mirror of scalars
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // sequence number of the last ||r||^2 the CG loop asked the finalize kernel
  // to mirror into the pinned host scalars (it arrives with h_scal[S_HSEQ])
  double hseq = 0.0;
  // the right-hand side whose ||b||_W^2 is already in scal / h_scal[S_BN2]
  // (formed with the initial guess); the next CG solve of that b uses it
  const double* bn2_b = nullptr;
  // set with bn2_b when the iterate is zero and r (and, for the float32
  // V-cycle, r32) already holds that b: the next CG solve skips its first
  // true residual
  bool r_is_b = false;
  // Captured V-cycles (one hipGraphExec per operator / coefficient / options /
  // input buffer), replayed with a single launch; captured on cap_stream.
  struct VcGraph {
    int op, smoother, degree, rz, prec, z32;
    double c, ratio, omega;
    const void* b;
    hipGraphExec_t exec;
    double* result;
    int rz_parts;
  };
  std::vector<VcGraph> graphs;
  hipStream_t cap_stream = nullptr;
  bool use_graphs = true;
  // float32 CG search directions kept for batched iterate updates (ring_m
  // fields, 0: none; allocated on first use)
  float* ring[kRing] = {};
  int ring_m = -1;
  // CG with the float32 V-cycle: flexible (Polak-Ribiere) beta instead of
  // the plain one (BF_FLEX_BETA=1)
  bool flex_beta = false;
  // GMRES workspace (allocated on first use)
  int gm_m = 0;
  double* gm_V = nullptr;  // (m+1) vectors
  double* gm_Z = nullptr;  // m preconditioned vectors
  double* gm_y = nullptr;  // m coefficients (device)
  std::vector<void*> allocs;
  // bf_step runs the pressure half (independent of the Cahn-Hilliard half
  // within a step) on a second grid with its own stream and host thread, so
  // the two solves overlap (created on first use; BF_NO_OVERLAP=1 disables)
  bf_grid* twin = nullptr;
  hipStream_t twin_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool overlap = true;
  // Timing of the CG step kernel (bf_grid_cg_timing): a pair of events on the
  // stream around every cg_timing-th launch while recording is on (0: off);
  // the events are pooled and reused after each read.
  int cg_timing = 0;
  int64_t cg_count = 0;  // launches since recording started
  std::vector<hipEvent_t> cg_ev;   // pool, 2 per recorded launch
  std::vector<uint8_t> cg_first;   // per recorded launch: a first step of a Krylov cycle
  size_t cg_used = 0;              // events of the pool in use
  std::vector<hipEvent_t> ru_ev;   // the same for the residual update (k_r_update)
  size_t ru_used = 0;
};

namespace {

int dalloc(bf_grid* g, double** p, int64_t count) {
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, (size_t)count * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(BF_ENOMEM, "hipMalloc of %lld doubles failed: %s", (long long)count,
                hipGetErrorString(e));
  }
  g->allocs.push_back(ptr);
  *p = (double*)ptr;
  return BF_OK;
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// The float32 hierarchy and level-0 input of the mixed-precision V-cycle,
// allocated on first use (half the bytes of the float64 one).
// The ring of float32 search directions of CG with the float32 V-cycle: up
// to kRing fields within 1 GiB (4096^2: 16; 8192^2: 3; none above, or when
// the allocation fails: the CG step then updates x itself).  Returns ring_m.
int ensure_ring(bf_grid* g) {
  if (g->ring_m >= 0) return g->ring_m;
  const size_t field = sizeof(float) * (size_t)g->npts;
  int m = (int)std::min<size_t>(kRing, (size_t(1) << 30) / field);
  if (m < 3) m = 0;
  for (int i = 0; i < m; ++i) {
    void* ptr = nullptr;
    if (hipMalloc(&ptr, field) != hipSuccess) {
      (void)hipGetLastError();
      m = i;
      break;
    }
    g->allocs.push_back(ptr);
    g->ring[i] = (float*)ptr;
  }
  g->ring_m = m >= 3 ? m : 0;
  return g->ring_m;
}

int ensure_mixed(bf_grid* g) {
  if (g->r32) return BF_OK;
  std::vector<LevelT<float>> lv;
  auto fal = [&](float** p, int64_t cnt) -> int {
    void* ptr = nullptr;
    if (hipMalloc(&ptr, (size_t)cnt * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(BF_ENOMEM, "hipMalloc of %lld floats failed", (long long)cnt);
    }
    g->allocs.push_back(ptr);
    *p = (float*)ptr;
    return BF_OK;
  };
  for (const Level& D : g->lv) {
    LevelT<float> L;
    L.n = D.n;
    L.npts = D.npts;
    TRY(fal(&L.xa, L.npts));
    TRY(fal(&L.xb, L.npts));
    TRY(fal(&L.r, L.npts));
    TRY(fal(&L.b, L.npts));
    lv.push_back(L);
  }
  float* r32 = nullptr;
  float* z32 = nullptr;
  TRY(fal(&r32, g->npts));
  TRY(fal(&z32, g->npts));
  g->lvf = lv;
  g->r32 = r32;
  g->z32 = z32;
  return BF_OK;
}

// ------------------------------------------------------------ host-side small
// dense algebra for the coarsest grid (5 x 4 nodes).
int refl_h(int j, int n) {
  j = j < 0 ? -j : j;
  return j > n ? 2 * n - j : j;
}

// y = A x on an n-grid on the host (reflection in y, wrap in x).
void host_apply(int op, int n, double coef, const double* x, double* y) {
  auto X = [&](int j, int i) { return x[refl_h(j, n) * n + ((i % n) + n) % n]; };
  for (int j = 0; j <= n; ++j)
    for (int i = 0; i < n; ++i) {
      const double c = X(j, i);
      const double axis = X(j, i - 1) + X(j, i + 1) + X(j - 1, i) + X(j + 1, i);
      if (op == BF_OP_LAP) {
        y[j * n + i] = coef * (axis - 4.0 * c);
      } else if (op == BF_OP_HELM) {
        // wall rows are identity rows; interior rows read the wall rows as they are
        const double xm = (j >= 1) ? X(j - 1, i) : 0.0, xp = (j < n) ? X(j + 1, i) : 0.0;
        const double ax = X(j, i - 1) + X(j, i + 1) + xm + xp;
        y[j * n + i] = (j == 0 || j == n) ? c : c + coef * (4.0 * c - ax);
      } else {
        const double diag = X(j - 1, i - 1) + X(j - 1, i + 1) + X(j + 1, i - 1) + X(j + 1, i + 1);
        const double far = X(j, i - 2) + X(j, i + 2) + X(j - 2, i) + X(j + 2, i);
        y[j * n + i] = c + coef * (20.0 * c - 8.0 * axis + 2.0 * diag + far);
      }
    }
}

// In-place inverse of a size x size matrix by Gauss-Jordan with partial pivoting.
bool invert(std::vector<double>& M, int size) {
  std::vector<double> inv(size * size, 0.0);
  for (int k = 0; k < size; ++k) inv[k * size + k] = 1.0;
  for (int col = 0; col < size; ++col) {
    int piv = col;
    for (int r = col + 1; r < size; ++r)
      if (std::fabs(M[r * size + col]) > std::fabs(M[piv * size + col])) piv = r;
    if (M[piv * size + col] == 0.0) return false;
    if (piv != col)
      for (int c = 0; c < size; ++c) {
        std::swap(M[piv * size + c], M[col * size + c]);
        std::swap(inv[piv * size + c], inv[col * size + c]);
      }
    const double d = 1.0 / M[col * size + col];
    for (int c = 0; c < size; ++c) {
      M[col * size + c] *= d;
      inv[col * size + c] *= d;
    }
    for (int r = 0; r < size; ++r) {
      if (r == col) continue;
      const double f = M[r * size + col];
      if (f == 0.0) continue;
      for (int c = 0; c < size; ++c) {
        M[r * size + c] -= f * M[col * size + c];
        inv[r * size + c] -= f * inv[col * size + c];
      }
    }
  }
  M = inv;
  return true;
}

// Dense operator of the coarsest grid by probing with unit vectors.
std::vector<double> coarse_matrix(int op, double coef) {
  const int n = kCoarseN, size = kCoarseSize;
  std::vector<double> A(size * size), e(size), col(size);
  for (int l = 0; l < size; ++l) {
    std::fill(e.begin(), e.end(), 0.0);
    e[l] = 1.0;
    host_apply(op, n, coef, e.data(), col.data());
    for (int k = 0; k < size; ++k) A[k * size + l] = col[k];
  }
  return A;
}

// Exact coarsest-grid solution operators:
//  CH : G = A^{-1}
//  HELM: G = inverse of the interior block (rows 1..n-1), zero on the wall rows
//       and columns: the V-cycle's wall rows stay zero and whatever the
//       restriction leaves in the coarse wall rows is ignored
//  LAP: G = top-left block of [[L, 1], [w^T, 0]]^{-1}; G b solves L p = b - wmean(b)
//       with w^T p = 0 (the weighted-mean constraint on the null space).
int coarse_operator(int op, double c, std::vector<double>& G) {
  const int n = kCoarseN, size = kCoarseSize;
  if (op == BF_OP_CH) {
    G = coarse_matrix(op, c * std::pow((double)n, 4));
    if (!invert(G, size)) return fail(BF_EINVAL, "coarse Cahn-Hilliard matrix is singular");
  } else if (op == BF_OP_HELM) {
    const std::vector<double> A = coarse_matrix(op, c * (double)n * n);
    const int isz = (n - 1) * n;  // interior rows 1..n-1
    std::vector<double> B(isz * isz);
    for (int k = 0; k < isz; ++k)
      for (int l = 0; l < isz; ++l) B[k * isz + l] = A[(k + n) * size + (l + n)];
    if (!invert(B, isz)) return fail(BF_EINVAL, "coarse Helmholtz matrix is singular");
    G.assign(size * size, 0.0);
    for (int k = 0; k < isz; ++k)
      for (int l = 0; l < isz; ++l) G[(k + n) * size + (l + n)] = B[k * isz + l];
  } else {
    std::vector<double> A = coarse_matrix(op, (double)n * n);
    const int bs = size + 1;
    std::vector<double> B(bs * bs, 0.0);
    for (int k = 0; k < size; ++k) {
      for (int l = 0; l < size; ++l) B[k * bs + l] = A[k * size + l];
      B[k * bs + size] = 1.0;
      const int j = k / n;
      B[size * bs + k] = (j == 0 || j == n) ? 0.5 : 1.0;
    }
    if (!invert(B, bs)) return fail(BF_EINVAL, "coarse bordered Laplacian is singular");
    G.resize(size * size);
    for (int k = 0; k < size; ++k)
      for (int l = 0; l < size; ++l) G[k * size + l] = B[k * bs + l];
  }
  return BF_OK;
}

double* coarse_of(bf_grid* g, int op) {
  return op == BF_OP_CH ? g->coarse_ch : op == BF_OP_HELM ? g->coarse_helm : g->coarse_lap;
}

int upload_coarse(bf_grid* g, int op, double c) {
  const int size = kCoarseSize;
  std::vector<double> G;
  TRY(coarse_operator(op, c, G));
  double* dst = coarse_of(g, op);
  HIPCHK(hipMemcpyAsync(dst, G.data(), sizeof(double) * size * size, hipMemcpyHostToDevice,
                        g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  return BF_OK;
}

int ensure_coarse_ch(bf_grid* g, double c) {
  if (g->cached_c == c) return BF_OK;
  TRY(upload_coarse(g, BF_OP_CH, c));
  g->cached_c = c;
  return BF_OK;
}

int ensure_coarse_helm(bf_grid* g, double beta) {
  if (g->cached_beta == beta) return BF_OK;
  TRY(upload_coarse(g, BF_OP_HELM, beta));
  g->cached_beta = beta;
  return BF_OK;
}

// The coarsest-grid operator of op (CH and HELM for the coefficient last
// made current by ensure_coarse_*).
int ensure_coarse(bf_grid* g, int op, double c) {
  if (op == BF_OP_CH) return ensure_coarse_ch(g, c);
  if (op == BF_OP_HELM) return ensure_coarse_helm(g, c);
  return BF_OK;
}

// ------------------------------------------------------------ level operators
OpDesc level_op(int op, int n, double c) {
  OpDesc A;
  A.op = op;
  A.n = n;
  if (op == BF_OP_LAP) {
    A.coef = (double)n * (double)n;
    A.dinv_int = A.dinv_edge = -1.0 / (4.0 * A.coef);
  } else if (op == BF_OP_HELM) {
    A.coef = c * (double)n * (double)n;
    A.dinv_int = 1.0 / (1.0 + 4.0 * A.coef);
    A.dinv_edge = 0.0;  // wall rows: Dirichlet data, never smoothed
  } else if (op == kOpMob) {
    A.coef = c;  // the mobility field comes from the grid (g->mob)
    A.dinv_int = A.dinv_edge = 0.0;
  } else {
    const double s = c * std::pow((double)n, 4);
    A.coef = s;
    A.dinv_int = 1.0 / (1.0 + 20.0 * s);
    A.dinv_edge = 1.0 / (1.0 + 21.0 * s);
  }
  return A;
}

int nparts_of(const bf_grid* g) { return red_blocks(g->npts); }

struct Smoother {
  int degree = 0;
  double a[8] = {0};
  double g[8] = {0};
};

// Chebyshev iteration on [lmax/ratio, lmax] for D^{-1}A (three-term form;
// Saad, Iterative Methods for Sparse Linear Systems, Sec. 12.3.2), or damped
// Jacobi with weight omega.
Smoother make_smoother(int op, int n, double c, const bf_solver_opts& o) {
  Smoother S;
  S.degree = o.degree > 0 ? o.degree : (op == BF_OP_CH ? 3 : 2);
  if (o.smoother == BF_SMOOTH_JACOBI) {
    double w = o.omega;
    if (w <= 0) {
      if (op != BF_OP_CH) {
        w = 0.8;
      } else {
        const double s = c * std::pow((double)n, 4);
        w = 2.0 * (1.0 + 20.0 * s) / (2.0 + 68.0 * s);
      }
    }
    for (int k = 0; k < S.degree; ++k) {
      S.a[k] = w;
      S.g[k] = 0.0;
    }
    return S;
  }
  double lmax;
  if (op == BF_OP_LAP) {
    lmax = 2.0;
  } else if (op == BF_OP_HELM) {
    const double s = c * (double)n * n;
    lmax = (1.0 + 8.0 * s) / (1.0 + 4.0 * s);
  } else {
    const double s = c * std::pow((double)n, 4);
    lmax = (1.0 + 64.0 * s) / (1.0 + 20.0 * s);
  }
  const double ratio = o.ratio > 0 ? o.ratio : (op == BF_OP_CH ? 16.0 : 4.0);
  const double lmin = lmax / ratio;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  S.a[0] = 1.0 / theta;
  S.g[0] = 0.0;
  double rho = 1.0 / sigma;
  for (int k = 1; k < S.degree; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    S.a[k] = 2.0 * rn / delta;
    S.g[k] = rn * rho;
    rho = rn;
  }
  return S;
}

// One V-cycle on level l of hierarchy lv with right-hand side b (level 0:
// external pointer).  Returns the buffer holding the level's result.
//
// float64 hierarchy: if rz_parts is given (level 0 only) and the last
// smoothing sweep can produce it, that sweep also writes partials of
// <b, z>_W into g->partials and *rz_parts receives their count (0 when the
// caller must reduce <b, z>_W itself).
//
// float32 hierarchy (mixed precision): level 0 must be given zout, the
// float64 output, or (streamed level 0 only) zout32, a float32 one, and bd,
// the float64 right-hand side that b rounds.  The last sweep writes z into
// zout / zout32 and partials of <b, z>_W (first group) and <z, q>_W (second
// group, q = g->q) into g->partials; *rz_parts (if given) receives the group
// size.  Returns nullptr at level 0 (the result is zout / zout32).
template <typename T>
T* vcycle_level(bf_grid* g, std::vector<LevelT<T>>& lv, int op, double c,
                const bf_solver_opts& o, int l, const T* b, int* rz_parts = nullptr,
                double* zout = nullptr, const double* bd = nullptr,
                float* zout32 = nullptr) {
  constexpr bool F32 = std::is_same<T, float>::value;
  LevelT<T>& L = lv[l];
  hipStream_t st = g->stream;
  if (rz_parts) *rz_parts = 0;
  T* res = nullptr;
  if (L.n == kCoarseN) {
    launch_coarse_solve(kCoarseSize, coarse_of(g, op), b, L.xa, st);
    res = L.xa;
  } else if (L.n <= kTailTop) {
    // the rest of the cycle in one workgroup (fields in LDS)
    TailArgs P;
    P.nlev = 0;
    for (int n = L.n; n > kCoarseN; n /= 2) {
      const OpDesc A = level_op(op, n, c);
      const Smoother S = make_smoother(op, n, c, o);
      TailLevel& TL = P.lev[P.nlev++];
      TL.n = n;
      TL.degree = S.degree;
      TL.coef = A.coef;
      TL.dinv_int = A.dinv_int;
      TL.dinv_edge = A.dinv_edge;
      for (int k = 0; k < 8; ++k) {
        TL.a[k] = S.a[k];
        TL.g[k] = S.g[k];
      }
    }
    P.G = coarse_of(g, op);
    launch_tail(op, P, b, L.xa, st);
    res = L.xa;
  }
  if (res) {
    if constexpr (F32) {
      if (zout) {  // a float32 hierarchy this small: widen, then the two dots
        const int np = nparts_of(g);
        launch_to_double(L.npts, res, zout, st);
        launch_dot(L.n, bd, zout, g->partials, np, st);
        launch_dot(L.n, zout, g->q, g->partials + np, np, st);
        if (rz_parts) *rz_parts = np;
        return nullptr;
      }
    }
    return res;
  }
  const OpDesc A = level_op(op, L.n, c);
  const Smoother S = make_smoother(op, L.n, c, o);
  const bool streamed = stream_ok(L.n, (int)sizeof(T));
  const bool fused = streamed && S.degree >= 2;
  // pre-smoothing from zero
  T* cur = L.xa;
  T* oth = L.xb;
  bool have_r = false;  // the residual of the pre-smoothed iterate is in L.r
  // the fused passes take their coefficients from the arguments: single grids only
  const bool single = !g_batch.coef && g_batch.count <= 1;
  if (fused && S.degree == 3 && smooth3r_ok(L.n, (int)sizeof(T)) && single) {
    // all three sweeps and the residual in one pass (x1, x2 in registers)
    if constexpr (F32) {
      stream_smooth3_resid<T>(A, b, cur, L.r, S.a[0], S.a[1], S.g[1], S.a[2], S.g[2], st);
      have_r = true;
    }
  } else if (fused && S.degree == 2 && smooth3_ok(L.n) && single) {
    // both sweeps and the residual in one pass
    stream_smooth2_resid<T>(A, b, cur, L.r, S.a[0], S.a[1], S.g[1], st);
    have_r = true;
  } else if (fused && S.degree == 3 && smooth3_ok(L.n) && single) {
    // all three sweeps in one pass (x1 and x2 stay in registers)
    stream_smooth3_from_zero<T>(A, b, cur, S.a[0], S.a[1], S.g[1], S.a[2], S.g[2], st);
  } else if (fused) {
    // sweeps 0 and 1 in one pass (x1 = a0 D^-1 b is never stored), sweep 2
    // re-forms x1 from b for its (x - x_prev) term
    stream_smooth_from_zero<T>(A, b, cur, S.a[0], S.a[1], S.g[1], st);
    for (int k = 2; k < S.degree; ++k) {
      if (k == 2)
        stream_smooth_prev_from_b<T>(A, cur, b, oth, S.a[0], S.a[k], S.g[k], st);
      else
        launch_smooth<T>(A, cur, S.g[k] != 0.0 ? oth : nullptr, b, oth, S.a[k], S.g[k], st);
      std::swap(cur, oth);
    }
  } else {
    launch_smooth0<T>(A, b, cur, S.a[0], st);
    for (int k = 1; k < S.degree; ++k) {
      launch_smooth<T>(A, cur, (k == 1 || S.g[k] == 0.0) ? nullptr : oth, b, oth, S.a[k],
                       S.g[k], st);
      std::swap(cur, oth);
    }
  }
  // coarse-grid correction
  if (!have_r) launch_residual<T>(A, cur, b, L.r, nullptr, 0, st);
  LevelT<T>& C = lv[l + 1];
  launch_restrict<T>(L.n, L.r, C.b, st);
  T* e = vcycle_level<T>(g, lv, op, c, o, l + 1, C.b);
  if (streamed && single && post_ok(L.n, op, S.degree, S.g[0], (int)sizeof(T))) {
    // the correction and the whole post-smoother in one pass, into L.r
    const double pa[3] = {S.a[0], S.a[1], S.a[2]};
    const double pg[3] = {0.0, S.g[1], S.g[2]};
    if constexpr (F32) {
      if (zout32 || zout) {
        // <z, q>_W only for the flexible beta
        const double* qf = g->flex_beta ? g->q : nullptr;
        const int np = zout32 ? stream_post_dot2_f32(A, S.degree, cur, e, b, zout32, qf, pa, pg,
                                                     g->partials, st)
                              : stream_post_dot2(A, S.degree, cur, e, b, zout, qf, pa, pg,
                                                 g->partials, st);
        if (rz_parts) *rz_parts = np;
        return nullptr;
      }
    } else {
      if (rz_parts) {
        *rz_parts = stream_post_dot(A, S.degree, cur, e, b, L.r, pa, pg, g->partials, st);
        return L.r;
      }
    }
    stream_post<T>(A, S.degree, cur, e, b, L.r, pa, pg, st);
    return L.r;
  }
  if constexpr (!F32) {
    if (streamed && single && smooth_last2_ok(L.n) && post1_ok(L.n, op, S.degree, S.g[0])) {
      // the correction and the first post-sweep in one pass (x1 into oth, x0 =
      // x + P e into L.r, free after the restriction), then the last two
      // sweeps in one pass, into cur (x is no longer read)
      stream_post1<T>(A, cur, e, b, oth, L.r, S.a[0], st);
      if (rz_parts) {
        *rz_parts = stream_smooth_last2_dot(A, oth, L.r, b, cur, S.a[1], S.g[1], S.a[2], S.g[2],
                                            g->partials, st);
        return cur;
      }
      stream_smooth_last2<T>(A, oth, L.r, b, cur, S.a[1], S.g[1], S.a[2], S.g[2], st);
      return cur;
    }
  }
  launch_prolong_add<T>(L.n, e, cur, st);
  // post-smoothing (same polynomial); on streamed single grids the last two
  // sweeps run as one pass, whose result goes to L.r (free on the way up:
  // the pass still reads the two previous iterates)
  const bool pair = streamed && S.degree >= 2 && smooth_last2_ok(L.n) && single;
  for (int k = 0; k < S.degree; ++k) {
    if (pair && k == S.degree - 2) {
      const int k2 = k + 1;
      if constexpr (F32) {
        if (zout32 || zout) {
          const int np =
              zout32 ? stream_smooth_last2_dot2_f32(A, cur, oth, b, zout32, g->q, S.a[k], S.g[k],
                                                    S.a[k2], S.g[k2], g->partials, st)
                     : stream_smooth_last2_dot2(A, cur, oth, b, zout, g->q, S.a[k], S.g[k],
                                                S.a[k2], S.g[k2], g->partials, st);
          if (rz_parts) *rz_parts = np;
          return nullptr;
        }
      } else {
        if (rz_parts) {
          *rz_parts = stream_smooth_last2_dot(A, cur, oth, b, L.r, S.a[k], S.g[k], S.a[k2],
                                              S.g[k2], g->partials, st);
          return L.r;
        }
      }
      stream_smooth_last2<T>(A, cur, oth, b, L.r, S.a[k], S.g[k], S.a[k2], S.g[k2], st);
      return L.r;
    }
    const T* prev = S.g[k] != 0.0 ? oth : nullptr;
    const bool last = k == S.degree - 1;
    if constexpr (F32) {
      if (last && (zout || zout32)) {
        int np;
        if (streamed && zout32) {
          np = stream_smooth_dot2_f32(A, cur, prev, b, zout32, g->q, S.a[k], S.g[k], g->partials,
                                      st);
        } else if (streamed) {
          np = stream_smooth_dot2(A, cur, prev, b, zout, g->q, S.a[k], S.g[k], g->partials, st);
        } else {
          np = nparts_of(g);
          launch_smooth<T>(A, cur, prev, b, oth, S.a[k], S.g[k], st);
          launch_to_double(L.npts, oth, zout, st);
          launch_dot(L.n, bd, zout, g->partials, np, st);
          launch_dot(L.n, zout, g->q, g->partials + np, np, st);
        }
        if (rz_parts) *rz_parts = np;
        return nullptr;
      }
      launch_smooth<T>(A, cur, prev, b, oth, S.a[k], S.g[k], st);
    } else {
      if (rz_parts && last && streamed)
        *rz_parts = stream_smooth_dot(A, cur, prev, b, oth, S.a[k], S.g[k], g->partials, st);
      else
        launch_smooth<T>(A, cur, prev, b, oth, S.a[k], S.g[k], st);
    }
    std::swap(cur, oth);
  }
  return cur;
}

// The V-cycle from level 0 in the precision o.mg_precision selects; the
// float32 cycle reads g->r32 (already holding the rounded r) and writes z
// into g->z.  Returns the buffer holding z.
double* vcycle_top(bf_grid* g, int op, double c, const bf_solver_opts& o, const double* r,
                   int* rz_parts) {
  if (o.mg_precision == BF_MG_F32) {
    vcycle_level<float>(g, g->lvf, op, c, o, 0, g->r32, rz_parts, g->want_z32 ? nullptr : g->z,
                        r, g->want_z32 ? g->z32 : nullptr);
    return g->z;
  }
  return vcycle_level<double>(g, g->lv, op, c, o, 0, r, rz_parts);
}

// Node mobilities of every level above the coarse tail (level 0: m itself,
// then injection), for the variable-mobility V-cycle; allocated on first use.
template <typename T>
int setup_mob_levels(bf_grid* g, std::vector<LevelT<T>>& lv, const double* m) {
  for (size_t l = 0; l < lv.size() && lv[l].n > kTailTop; ++l) {
    if (!lv[l].m) {
      void* ptr = nullptr;
      if (hipMalloc(&ptr, sizeof(T) * (size_t)lv[l].npts) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BF_ENOMEM, "mobility level allocation failed");
      }
      g->allocs.push_back(ptr);
      lv[l].m = (T*)ptr;
    }
  }
  if (lv.empty() || lv[0].n <= kTailTop) return BF_OK;
  if constexpr (std::is_same<T, float>::value)
    launch_to_float(lv[0].npts, m, lv[0].m, g->stream);
  else
    launch_copy(lv[0].npts, m, lv[0].m, g->stream);
  for (size_t l = 0; l + 1 < lv.size() && lv[l + 1].n > kTailTop; ++l)
    launch_inject<T>(lv[l].n, lv[l].m, lv[l + 1].m, g->stream);
  return BF_OK;
}

// One V-cycle of the variable-mobility operator I + c L_m L from level l:
// on every level above the coarse tail the operator is rediscretised with the
// level's mobilities (smoothing and residual by the k_mob_* kernels, the same
// Chebyshev polynomial as the constant-mobility cycle at the mean mobility);
// the tail and the exact coarsest solve use the constant mean mobility.
template <typename T>
T* vcycle_mob(bf_grid* g, std::vector<LevelT<T>>& lv, double c, const bf_solver_opts& o, int l,
              const T* b) {
  LevelT<T>& L = lv[l];
  if (L.n <= kTailTop) return vcycle_level<T>(g, lv, BF_OP_CH, c * g->mob_pre, o, l, b);
  hipStream_t st = g->stream;
  const double cs = c * std::pow((double)L.n, 4);
  const Smoother S = make_smoother(BF_OP_CH, L.n, c * g->mob_pre, o);
  T* cur = L.xa;
  T* oth = L.xb;
  launch_mob_smooth0<T>(L.n, cs, L.m, b, cur, S.a[0], st);
  for (int k = 1; k < S.degree; ++k) {
    launch_mob_smooth<T>(L.n, cs, L.m, cur, (k == 1 || S.g[k] == 0.0) ? nullptr : oth, b, oth,
                         S.a[k], S.g[k], st);
    std::swap(cur, oth);
  }
  launch_mob_residual<T>(L.n, cs, L.m, cur, b, L.r, st);
  LevelT<T>& C = lv[l + 1];
  launch_restrict<T>(L.n, L.r, C.b, st);
  T* e = vcycle_mob<T>(g, lv, c, o, l + 1, C.b);
  launch_prolong_add<T>(L.n, e, cur, st);
  for (int k = 0; k < S.degree; ++k) {
    launch_mob_smooth<T>(L.n, cs, L.m, cur, S.g[k] != 0.0 ? oth : nullptr, b, oth, S.a[k],
                         S.g[k], st);
    std::swap(cur, oth);
  }
  return cur;
}

int check_opts(const bf_solver_opts& o) {
  if (o.ksp != BF_KSP_CG && o.ksp != BF_KSP_GMRES) return fail(BF_EINVAL, "ksp %d", o.ksp);
  if (o.pc < BF_PC_NONE || o.pc > BF_PC_MG) return fail(BF_EINVAL, "pc %d", o.pc);
  if (o.maxit < 1) return fail(BF_EINVAL, "maxit %d < 1", o.maxit);
  if (o.degree < 0 || o.degree > 8) return fail(BF_EINVAL, "degree %d not in 0..8", o.degree);
  if (o.smoother != BF_SMOOTH_CHEBYSHEV && o.smoother != BF_SMOOTH_JACOBI)
    return fail(BF_EINVAL, "smoother %d", o.smoother);
  if (!(o.rtol > 0)) return fail(BF_EINVAL, "rtol must be > 0");
  if (o.ksp == BF_KSP_GMRES && (o.restart < 1 || o.restart > 64))
    return fail(BF_EINVAL, "restart %d not in 1..64", o.restart);
  if (o.check_every < 1) return fail(BF_EINVAL, "check_every %d < 1", o.check_every);
  if (o.ratio < 0 || o.omega < 0) return fail(BF_EINVAL, "negative ratio/omega");
  if (o.mg_precision != BF_MG_F64 && o.mg_precision != BF_MG_F32)
    return fail(BF_EINVAL, "mg_precision %d", o.mg_precision);
  return BF_OK;
}

// The V-cycle from level 0 as a replayed HIP graph.  The whole cycle (about
// 7 launches per level above the tail) is captured once per (operator, c,
// smoother options, input buffer, <b,z> fusion) on the grid's private capture
// stream and launched on the grid's stream with one call: on the coarse
// levels the kernels are shorter than the host's per-launch cost, so eager
// launches left the GPU idle between them.  Returns nullptr if capture is
// unavailable (the caller then launches eagerly).
double* vcycle_graph(bf_grid* g, int op, double c, const bf_solver_opts& o, const double* b,
                     int* rz_parts) {
  const int rz = rz_parts ? 1 : 0;
  for (auto& e : g->graphs) {
    if (e.op == op && e.c == c && e.smoother == o.smoother && e.degree == o.degree &&
        e.ratio == o.ratio && e.omega == o.omega && e.b == b && e.rz == rz &&
        e.prec == o.mg_precision && e.z32 == (g->want_z32 ? 1 : 0)) {
      if (hipGraphLaunch(e.exec, g->stream) != hipSuccess) return nullptr;
      if (rz_parts) *rz_parts = e.rz_parts;
      return e.result;
    }
  }
  if (g->graphs.size() >= 96) {
    (void)hipGraphExecDestroy(g->graphs.front().exec);
    g->graphs.erase(g->graphs.begin());
  }
  bf_grid::VcGraph e;
  e.op = op;
  e.c = c;
  e.smoother = o.smoother;
  e.degree = o.degree;
  e.ratio = o.ratio;
  e.omega = o.omega;
  e.b = b;
  e.rz = rz;
  e.prec = o.mg_precision;
  e.z32 = g->want_z32 ? 1 : 0;
  e.rz_parts = 0;
  hipStream_t user = g->stream;
  if (hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  g->stream = g->cap_stream;
  e.result = vcycle_top(g, op, c, o, b, rz ? &e.rz_parts : nullptr);
  g->stream = user;
  hipGraph_t graph = nullptr;
  if (hipStreamEndCapture(g->cap_stream, &graph) != hipSuccess || !graph) {
    (void)hipGetLastError();
    return nullptr;
  }
  const hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  g->graphs.push_back(e);
  if (hipGraphLaunch(e.exec, g->stream) != hipSuccess) return nullptr;
  if (rz_parts) *rz_parts = e.rz_parts;
  return e.result;
}

// z = M r for the chosen preconditioner.  Returns the buffer holding z; see
// vcycle_level for rz_parts.  With the float32 V-cycle, r32_ready says that
// g->r32 already holds (float) r (the CG residual update writes it).
double* precondition(bf_grid* g, int op, double c, const bf_solver_opts& o, const double* r,
                     int* rz_parts = nullptr, bool r32_ready = false) {
  if (rz_parts) *rz_parts = 0;
  switch (o.pc) {
    case BF_PC_MG:
      if (o.mg_precision == BF_MG_F32 && !r32_ready) launch_to_float(g->npts, r, g->r32, g->stream);
      if (g->use_graphs) {
        double* z = vcycle_graph(g, op, c, o, r, rz_parts);
        if (z) return z;
        g->use_graphs = false;  // capture not available: launch eagerly from now on
      }
      return vcycle_top(g, op, c, o, r, rz_parts);
    case BF_PC_JACOBI:
      launch_jacobi_pc(level_op(op, g->n, c), r, g->z, g->stream);
      return g->z;
    default:
      launch_copy(g->npts, r, g->z, g->stream);
      return g->z;
  }
}

// z = M r for the variable-mobility operator: the variable-mobility V-cycle
// (multigrid), else the constant-mobility preconditioner at the mean mobility.
double* precondition_mob(bf_grid* g, double c, const bf_solver_opts& o, const double* r) {
  if (o.pc != BF_PC_MG) return precondition(g, BF_OP_CH, c * g->mob_pre, o, r);
  if (o.mg_precision == BF_MG_F32) {
    launch_to_float(g->npts, r, g->r32, g->stream);
    float* zf = vcycle_mob<float>(g, g->lvf, c, o, 0, g->r32);
    launch_to_double(g->npts, zf, g->z, g->stream);
    return g->z;
  }
  return vcycle_mob<double>(g, g->lv, c, o, 0, r);
}

// Start the timing of one CG-step launch: takes a pair of events from the
// pool (creating them on first use) and records the first on the stream; the
// caller records the second after the launch.
// A pair of events from the pool (created on demand): the first is recorded now,
// the caller records the second after the launch.
int timing_pair(bf_grid* g, std::vector<hipEvent_t>& pool, size_t& used) {
  if (used + 2 > pool.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e = nullptr;
      HIPCHK(hipEventCreate(&e));
      pool.push_back(e);
    }
  }
  HIPCHK(hipEventRecord(pool[used], g->stream));
  used += 2;
  return BF_OK;
}

int cg_timing_mark(bf_grid* g, bool first) {
  if (g->cg_used + 2 > g->cg_ev.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e = nullptr;
      HIPCHK(hipEventCreate(&e));
      g->cg_ev.push_back(e);
    }
  }
  HIPCHK(hipEventRecord(g->cg_ev[g->cg_used], g->stream));
  g->cg_used += 2;
  g->cg_first.push_back(first ? 1 : 0);
  return BF_OK;
}

// Reduce <x, y>_W into scal[slot] (asynchronous).
void wdot_async(bf_grid* g, const double* x, const double* y, int mode, int slot) {
  const int np = nparts_of(g);
  launch_dot(g->n, x, y, g->partials, np, g->stream);
  launch_finalize(g->partials, np, g->scal, mode, slot, g->n, g->stream);
}

int read_scalars(bf_grid* g, int count) {
  HIPCHK(hipMemcpyAsync(g->h_scal, g->scal, sizeof(double) * count, hipMemcpyDeviceToHost,
                        g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  return BF_OK;
}

// Wait until the finalize that mirrors its value into the pinned host scalars
// with sequence number g->hseq has done so (work queued behind it keeps the GPU
// busy while the host waits).  The kernel writes the value, then the number,
// each followed by a system-scope fence, so the value is visible once the
// number is.  An event recorded on the stream for this would leave the stream
// idle for about 5 us per wait.  If the stream drains without the number
// arriving, the wait fails instead of spinning on.
int wait_scalars(bf_grid* g) {
  const volatile double* seq = g->h_scal + S_HSEQ;
  for (uint64_t spin = 1;; ++spin) {
    if (*seq == g->hseq) break;
    if ((spin & 0xffff) == 0) {
      const hipError_t q = hipStreamQuery(g->stream);
      if (q == hipSuccess) {
        if (*seq == g->hseq) break;
        return fail(BF_EHIP, "the residual norm did not reach the host");
      }
      if (q != hipErrorNotReady) HIPCHK(q);
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return BF_OK;
}

// Constant-mode (mass) correction of a Cahn-Hilliard iterate.  The constant
// field is an eigenvector of I + c L^2 with eigenvalue 1 and sum_W L^2 x = 0,
// so the exact solution has sum_W x = sum_W b.  Adding the weighted mean of
// (b - x) removes the constant-mode error of x (mass is then conserved to
// rounding) and can only lower ||b - A x||_W.  The sums are taken on b and x
// directly, not on a residual whose rounding is amplified by c/h^4.
void mass_correct(bf_grid* g, const double* b, double* x) {
  const int np = nparts_of(g);
  launch_wsum_diff(g->n, b, x, g->partials, np, g->stream);
  launch_finalize(g->partials, np, g->scal, F_MEAN, 0, g->n, g->stream);
  launch_add_mean(g->n, x, x, g->scal, g->stream);
}

// ------------------------------------------------------------ Krylov drivers
// Final status from the true residual (residual replacement / floor logic).
struct KrylovState {
  int iters = 0, restarts = 0;
  int x_updates = 0;  // rounded additions the iterate went through (see floor_accept)
  double rel = 0, rel_true = 0, floor_est = 0;
  double rel_est_cycle = HUGE_VAL;  // GMRES: residual estimate at the end of a cycle
};

// Sum over j of A_jk^2 for an interior column k of the operator (the
// amplification of independent rounding errors of x into the residual).
double column_sq(const OpDesc& A) {
  if (A.op == BF_OP_LAP) return 20.0 * A.coef * A.coef;
  if (A.op == BF_OP_HELM) return (1.0 + 4.0 * A.coef) * (1.0 + 4.0 * A.coef) + 4.0 * A.coef * A.coef;
  const double d = 1.0 + 20.0 * A.coef;
  return d * d + 276.0 * A.coef * A.coef;
}

// True residual r = b - A x with the double-double stencil sum, written into r;
// returns (via ks) ||r||_W / ||b||_W and the expected float64 representation
// floor of that quantity, sqrt(sum_W ulp(x)^2 / 12 * column_sq) / ||b||_W.
// r32 (optional): where the tiled kernel runs, it also writes (float) r there
// and *r32_done says so (the float32 V-cycle's input, without a separate pass).
int true_residual(bf_grid* g, const OpDesc& A, const double* b, const double* x, double* r,
                  double bn, KrylovState& ks, float* r32 = nullptr, bool* r32_done = nullptr) {
  const int np = nparts_of(g);
  const bool fused32 = r32 && A.op != kOpMob && stream_ok(g->n);
  if (r32_done) *r32_done = fused32;
  const int nr = A.op == kOpMob
                     ? launch_mob(g->n, A.coef, g->mob, x, b, r, g->partials, np, g->stream)
                 : fused32 ? stream_residual_dd(A, x, b, r, g->partials, g->stream, r32)
                           : launch_residual_dd(A, x, b, r, g->partials, np, g->stream);
  launch_finalize(g->partials, nr, g->scal, F_STORE, S_RTRUE, g->n, g->stream);
  launch_finalize(g->partials + nr, nr, g->scal, F_STORE, S_ULP2, g->n, g->stream);
  TRY(read_scalars(g, S_ULP2 + 1));
  ks.rel_true = std::sqrt(g->h_scal[S_RTRUE]) / bn;
  // (variable mobility: the kernel already weights ulp(x)^2 by the local column sum)
  const double csq = A.op == kOpMob ? 1.0 : column_sq(A);
  ks.floor_est = std::sqrt(g->h_scal[S_ULP2] / 12.0 * csq) / bn;
  if (!std::isfinite(ks.rel_true)) return fail(BF_ENONFINITE, "true residual is not finite");
  return BF_OK;
}

// After a Krylov cycle has driven its recursive residual to rtol: decide from
// the true residual whether to stop (BF_OK / BF_AT_FLOOR / BF_NOT_CONVERGED)
// or to restart from it (returns -1 = restart).
//  - true residual <= rtol: converged;
//  - true residual within the floor bound of the iterate (floor_accept: the
//    rounding noise of an iterate built by ks.x_updates rounded additions),
//    BF_AT_FLOOR: no float64 vector formed that way does much better, and the
//    recursive residual, which does not see that rounding, met rtol;
//  - otherwise restart (iterative refinement) while each restart at least
//    halves the true residual, up to max_restarts;
//  - a restart that stops improving within twice the floor bound is also
//    BF_AT_FLOOR;
//  - else BF_NOT_CONVERGED.
int decide_after_cycle(const bf_solver_opts& o, KrylovState& ks, double& last_true,
                       bool hit_maxit) {
  if (ks.rel_true <= o.rtol) return BF_OK;
  if (hit_maxit) return BF_NOT_CONVERGED;
  const double fb = floor_accept(ks.floor_est, ks.x_updates);
  if (ks.rel_true <= fb) return BF_AT_FLOOR;
  if (ks.restarts < o.max_restarts && ks.rel_true < 0.5 * last_true) {
    ks.restarts++;
    last_true = ks.rel_true;
    return -1;
  }
  return ks.rel_true <= 2.0 * fb ? BF_AT_FLOOR : BF_NOT_CONVERGED;
}

// Residual norms of a CG cycle, for deciding when the host may read the next
// norm late.  A synchronous read idles the GPU for the copy, the host's
// wake-up and the launch of the next kernels (about 35 us, against about
// 1 ms per iteration at 4096^2).  While the next norm is predicted to stay
// well above rtol, the host queues the next preconditioner application
// first and reads the norm while it runs.  The prediction extrapolates the
// last known norm with the fastest per-iteration reduction seen in the cycle
// (0.1 before two norms are known); a wrong guess costs one preconditioner
// application that is discarded.
struct NormTrack {
  int k_last = 0;
  double rel_last = 0.0;
  double fastest = 0.1;
  bool have_ratio = false;
  double predict(int k) const { return rel_last * std::pow(fastest, k - k_last); }
  void take(int k, double rel) {
    if (k > k_last && rel_last > 0.0 && rel > 0.0) {
      const double r = std::pow(rel / rel_last, 1.0 / (k - k_last));
      fastest = have_ratio ? std::min(fastest, r) : r;
      have_ratio = true;
    }
    k_last = k;
    rel_last = rel;
  }
};

// CG in the weighted inner product.  For the Cahn-Hilliard operator q = A p
// is evaluated with the double-double stencil sum, so the recursive residual
// tracks the true one up to the rounding of x itself.  Whenever the recursive
// residual reaches rtol the true residual is recomputed (double-double) and
// decide_after_cycle() stops or restarts from it (residual replacement, i.e.
// iterative refinement).
int run_cg(bf_grid* g, int op, double c, const double* b, double* x, const bf_solver_opts& o,
           KrylovState& ks, bool bn2_known, bool r_is_b) {
  hipStream_t st = g->stream;
  const int np = nparts_of(g);
  const OpDesc A = level_op(op, g->n, c);
  double bn2;
  if (bn2_known) {
    bn2 = g->h_scal[S_BN2];  // formed with the initial guess (ch_guess)
  } else {
    wdot_async(g, b, b, F_STORE, S_BN2);
    TRY(read_scalars(g, S_BN2 + 1));
    bn2 = g->h_scal[S_BN2];
  }
  if (!std::isfinite(bn2)) return fail(BF_ENONFINITE, "right-hand side is not finite");
  if (bn2 == 0.0) {
    launch_fill(g->npts, x, 0.0, st);
    ks.rel = ks.rel_true = 0.0;
    return BF_OK;
  }
  const double bn = std::sqrt(bn2);
  // The float32 V-cycle is a symmetric positive definite operator up to
  // rounding (the same Chebyshev polynomial before and after the coarse
  // correction, restriction the weighted adjoint of the interpolation), so
  // beta = rho_k / rho_{k-1} as with the float64 one: the flexible
  // (Polak-Ribiere) form -alpha <z_k, q_{k-1}>_W / rho_{k-1}, for
  // preconditioners that vary from one application to the next, took the
  // same iterations at 4096^2 (14.3 and 8.0 per step) and costs the top
  // post-smoothing pass a read of q (BF_FLEX_BETA=1 selects it).
  const bool mixed = o.pc == BF_PC_MG && o.mg_precision == BF_MG_F32;
  if (mixed) TRY(ensure_mixed(g));
  // the true residual also writes (float) r for the first float32 V-cycle
  bool r32_ready = false;
  if (r_is_b) {
    // x = 0 and r = b - A 0 = b is in place (solve_pressure_zero)
    ks.rel_true = 1.0;
    ks.floor_est = 0.0;
    r32_ready = mixed;
  } else {
    TRY(true_residual(g, A, b, x, g->r, bn, ks, mixed ? g->r32 : nullptr, &r32_ready));
  }
  ks.rel = ks.rel_true;
  if (ks.rel_true <= o.rtol) return BF_OK;
  double last_true = ks.rel_true;
  // streamed top level: the float32 V-cycle hands z over in float32 (z32)
  const bool zf32 = mixed && stream_ok(g->n, 4);
  struct Z32Scope {
    bf_grid* g;
    ~Z32Scope() { g->want_z32 = false; }
  } z32_scope{g};
  g->want_z32 = zf32;
  // search directions (float32 when z is: stream_cg_p32)
  double* pcur = g->p;
  double* pnext = g->p2;
  // With the float32 directions in the ring, the CG step leaves x alone and
  // x += sum alpha_i p_i runs once per ring_m steps (x is read and written
  // once per batch instead of once per step; p_i is read once more).
  const int rm = zf32 ? ensure_ring(g) : 0;
  for (;;) {
    // (re)start from the residual in g->r
    int rzp = 0;
    double* z = precondition(g, op, c, o, g->r, &rzp, r32_ready);
    if (rzp > 0)
      launch_finalize(g->partials, rzp, g->scal, F_STORE, S_RZ, g->n, st);
    else
      wdot_async(g, g->r, z, F_STORE, S_RZ);
    bool first = true;     // p = z (no beta term, no pending x update)
    bool pending = false;  // x still lacks alpha * pcur
    int head = 0;          // ring: slot of the next direction
    int nring = 0;         // ring: directions whose x update is pending
    auto flush_ring = [&]() {
      const float* ps[kRing];
      for (int i = 0; i < nring; ++i) ps[i] = g->ring[(head - nring + i + rm) % rm];
      launch_x_accum(g->n, x, ps, nring, g->scal + S_AHIST, st);
      nring = 0;
    };
    bool converged = false;
    NormTrack nt;
    nt.take(ks.iters, ks.rel_true);
    auto take_norm = [&]() -> int {
      ks.rel = std::sqrt(g->h_scal[S_RR]) / bn;
      if (!std::isfinite(ks.rel)) return fail(BF_ENONFINITE, "residual norm is not finite");
      nt.take(ks.iters, ks.rel);
      return ks.rel <= o.rtol ? 1 : 0;
    };
    while (ks.iters < o.maxit) {
      // p' = z + beta p, q = A p' (+ <p', q>), and the deferred x += alpha p
      const bool timed = g->cg_timing > 0 && op == BF_OP_CH && g->cg_count++ % g->cg_timing == 0;
      if (timed) TRY(cg_timing_mark(g, first));
      int npq;
      if (rm) {
        if (nring == rm) flush_ring();
        npq = stream_cg_p32(A, g->z32, first ? nullptr : g->ring[(head + rm - 1) % rm],
                            g->ring[head], g->q, nullptr, g->scal, first, g->partials, st);
      } else {
        npq = zf32 ? stream_cg_p32(A, g->z32, reinterpret_cast<const float*>(pcur),
                                   reinterpret_cast<float*>(pnext), g->q, x, g->scal, first,
                                   g->partials, st)
                   : launch_cg_p(A, z, pcur, pnext, g->q, x, g->scal, first, g->partials, np, st);
      }
      if (timed) HIPCHK(hipEventRecord(g->cg_ev[g->cg_used - 1], st));
      launch_finalize(g->partials, npq, g->scal, F_ALPHA, rm ? S_AHIST + nring : 0, g->n, st);
      if (rm) {
        head = (head + 1) % rm;
        nring++;
      } else {
        std::swap(pcur, pnext);
        pending = true;
      }
      first = false;
      if (timed) TRY(timing_pair(g, g->ru_ev, g->ru_used));
      launch_r_update(g->n, g->r, g->q, g->scal, g->partials, np, st, mixed ? g->r32 : nullptr);
      if (timed) HIPCHK(hipEventRecord(g->ru_ev[g->ru_used - 1], st));
      // ||r||^2 also lands in the pinned host scalars: an event then says it arrived
      g->hseq += 1.0;
      launch_finalize(g->partials, np, g->scal, F_STORE, S_RR, g->n, st, g->h_scal, g->hseq);
      ks.iters++;
      ks.x_updates++;
      bool deferred = false;
      if (ks.iters % o.check_every == 0 || ks.iters == o.maxit) {
        deferred = ks.iters < o.maxit && nt.predict(ks.iters) > 4.0 * o.rtol;
        if (!deferred) {
          TRY(wait_scalars(g));
          const int t = take_norm();
          if (t < 0) return t;
          if (t > 0) {
            converged = true;
            break;
          }
        }
      }
      z = precondition(g, op, c, o, g->r, &rzp, mixed);
      if (mixed && g->flex_beta)
        launch_finalize_flex(g->partials, rzp, g->scal, st);
      else if (rzp > 0)
        launch_finalize(g->partials, rzp, g->scal, F_BETA, 0, g->n, st);
      else
        wdot_async(g, g->r, z, F_BETA, 0);
      if (deferred) {
        // the norm of this iteration arrives while the preconditioner runs; if
        // it already meets rtol that application is not used (it changes z and
        // the beta scalars only, not alpha or the iterate)
        TRY(wait_scalars(g));
        const int t = take_norm();
        if (t < 0) return t;
        if (t > 0) {
          converged = true;
          break;
        }
      }
    }
    if (nring > 0) flush_ring();
    if (pending) {
      if (zf32)
        launch_x_update(g->n, x, reinterpret_cast<const float*>(pcur), g->scal, st);
      else
        launch_x_update(g->n, x, pcur, g->scal, st);
    }
    if (op == BF_OP_CH) {
      mass_correct(g, b, x);
      ks.x_updates++;
    }
    TRY(true_residual(g, A, b, x, g->r, bn, ks, mixed ? g->r32 : nullptr, &r32_ready));
    const int d = decide_after_cycle(o, ks, last_true, !converged);
    if (d >= 0) return d;
  }
}

int ensure_gmres(bf_grid* g, int m) {
  if (g->gm_m >= m) return BF_OK;
  if (g->gm_V) {
    HIPCHK(hipFree(g->gm_V));
    HIPCHK(hipFree(g->gm_Z));
    HIPCHK(hipFree(g->gm_y));
    for (auto& p : g->allocs)
      if (p == g->gm_V || p == g->gm_Z || p == g->gm_y) p = nullptr;
    g->gm_V = g->gm_Z = g->gm_y = nullptr;
    g->gm_m = 0;
  }
  TRY(dalloc(g, &g->gm_V, (int64_t)(m + 1) * g->npts));
  TRY(dalloc(g, &g->gm_Z, (int64_t)m * g->npts));
  TRY(dalloc(g, &g->gm_y, m));
  g->gm_m = m;
  return BF_OK;
}

// Right-preconditioned (flexible) GMRES(m) in the weighted inner product with
// classical Gram-Schmidt applied twice; Givens rotations on the host.
int run_gmres(bf_grid* g, int op, double c, const double* b, double* x, const bf_solver_opts& o,
              KrylovState& ks) {
  hipStream_t st = g->stream;
  const int np = nparts_of(g);
  const int m = o.restart;
  TRY(ensure_gmres(g, m));
  if (o.pc == BF_PC_MG && o.mg_precision == BF_MG_F32) TRY(ensure_mixed(g));
  const OpDesc A = level_op(op, g->n, c);
  const int64_t N = g->npts;
  wdot_async(g, b, b, F_STORE, S_BN2);
  TRY(read_scalars(g, S_BN2 + 1));
  const double bn2 = g->h_scal[S_BN2];
  if (!std::isfinite(bn2)) return fail(BF_ENONFINITE, "right-hand side is not finite");
  if (bn2 == 0.0) {
    launch_fill(g->npts, x, 0.0, st);
    return BF_OK;
  }
  const double bn = std::sqrt(bn2);
  std::vector<double> H((m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
  double last_true = HUGE_VAL;
  for (int cycle = 0;; ++cycle) {
    // r0 = b - A x (double-double), V0 = r0 / ||r0||
    if ((op == BF_OP_CH || op == kOpMob) && cycle > 0) {
      mass_correct(g, b, x);
      ks.x_updates++;
    }
    TRY(true_residual(g, A, b, x, g->gm_V, bn, ks));
    ks.rel = ks.rel_true;
    if (cycle == 0) {
      if (ks.rel_true <= o.rtol) return BF_OK;
      last_true = ks.rel_true;
    } else {
      // a GMRES cycle ends at rtol (estimated) or after m steps; only the
      // former is a converged cycle for decide_after_cycle()
      const bool cycle_converged = ks.rel_est_cycle <= o.rtol;
      if (cycle_converged || ks.iters >= o.maxit) {
        const int d = decide_after_cycle(o, ks, last_true, ks.iters >= o.maxit && !cycle_converged);
        if (d >= 0) return d;
      } else {
        if (ks.rel_true <= o.rtol) return BF_OK;
        last_true = std::min(last_true, ks.rel_true);
      }
    }
    const double beta = ks.rel_true * bn;
    launch_scale(g->n, g->gm_V, g->gm_V, g->scal, S_RTRUE, 1, st);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    ks.rel_est_cycle = HUGE_VAL;
    int k = 0;
    for (; k < m && ks.iters < o.maxit; ++k) {
      double* Vk = g->gm_V + (int64_t)k * N;
      double* Zk = g->gm_Z + (int64_t)k * N;
      double* w = g->gm_V + (int64_t)(k + 1) * N;
      double* zk = op == kOpMob ? precondition_mob(g, c, o, Vk) : precondition(g, op, c, o, Vk);
      launch_copy(N, zk, Zk, st);
      if (op == kOpMob)
        launch_mob(g->n, c, g->mob, Zk, nullptr, w, nullptr, 0, st);
      else
        launch_apply_dot(A, Zk, w, g->partials, np, st, op == BF_OP_CH);
      // CGS2: h = V^T_W w, w -= V h, twice
      for (int pass = 0; pass < 2; ++pass) {
        launch_mdot(g->n, g->gm_V, k + 1, w, g->partials, np, st);
        launch_finalize_multi(g->partials, np, k + 1, g->scal, S_GM + pass * 72, st);
        launch_maxpy(g->n, g->gm_V, k + 1, g->scal + S_GM + pass * 72, w,
                     pass == 1 ? g->partials : nullptr, np, st);
      }
      launch_finalize(g->partials, np, g->scal, F_STORE, S_TMP, g->n, st);
      TRY(read_scalars(g, S_GM + 72 + k + 1));
      const double hn = std::sqrt(g->h_scal[S_TMP]);
      for (int i = 0; i <= k; ++i)
        H[i * m + k] = g->h_scal[S_GM + i] + g->h_scal[S_GM + 72 + i];
      H[(k + 1) * m + k] = hn;
      if (!std::isfinite(hn)) return fail(BF_ENONFINITE, "Arnoldi norm is not finite");
      if (hn > 0) launch_scale(g->n, w, w, g->scal, S_TMP, 1, st);
      // apply previous rotations, then a new one
      for (int i = 0; i < k; ++i) {
        const double t = cs[i] * H[i * m + k] + sn[i] * H[(i + 1) * m + k];
        H[(i + 1) * m + k] = -sn[i] * H[i * m + k] + cs[i] * H[(i + 1) * m + k];
        H[i * m + k] = t;
      }
      const double a = H[k * m + k], bb = H[(k + 1) * m + k];
      const double rr = std::hypot(a, bb);
      cs[k] = rr > 0 ? a / rr : 1.0;
      sn[k] = rr > 0 ? bb / rr : 0.0;
      H[k * m + k] = rr;
      H[(k + 1) * m + k] = 0.0;
      gv[k + 1] = -sn[k] * gv[k];
      gv[k] = cs[k] * gv[k];
      ks.iters++;
      ks.rel = std::fabs(gv[k + 1]) / bn;
      ks.rel_est_cycle = ks.rel;
      if (ks.rel <= o.rtol || hn == 0.0) {
        ++k;
        break;
      }
    }
    // y = H^{-1} g (upper triangular), x += Z y
    for (int i = k - 1; i >= 0; --i) {
      double s = gv[i];
      for (int j = i + 1; j < k; ++j) s -= H[i * m + j] * y[j];
      y[i] = s / H[i * m + i];
    }
    HIPCHK(hipMemcpyAsync(g->gm_y, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
    launch_axpy_multi(g->n, g->gm_Z, k, g->gm_y, x, st);
    ks.x_updates++;
    HIPCHK(hipStreamSynchronize(st));  // y is a host vector reused next cycle
  }
}

int run_krylov(bf_grid* g, int op, double c, const double* b, double* x, const bf_solver_opts& o,
               bf_solve_stats* st) {
  // ||b||_W^2 formed with the initial guess of this b (used once, by CG)
  const bool bn2_known = g->bn2_b == b;
  const bool r_is_b = bn2_known && g->r_is_b;
  g->bn2_b = nullptr;
  g->r_is_b = false;
  TRY(check_opts(o));
  if (op == kOpMob) {
    if (o.ksp != BF_KSP_GMRES)
      return fail(BF_EINVAL, "the variable-mobility operator is not symmetric: use GMRES");
    TRY(ensure_coarse(g, BF_OP_CH, c * g->mob_pre));
  } else {
    TRY(ensure_coarse(g, op, c));
  }
  HIPCHK(hipEventRecord(g->ev0, g->stream));
  if (op == BF_OP_HELM) {
    // Dirichlet walls: the iterate starts (and stays) at the wall data in b
    const size_t row = sizeof(double) * (size_t)g->n;
    HIPCHK(hipMemcpyAsync(x, b, row, hipMemcpyDeviceToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(x + (int64_t)g->n * g->n, b + (int64_t)g->n * g->n, row,
                          hipMemcpyDeviceToDevice, g->stream));
  }
  KrylovState ks;
  int status = o.ksp == BF_KSP_CG ? run_cg(g, op, c, b, x, o, ks, bn2_known, r_is_b)
                                  : run_gmres(g, op, c, b, x, o, ks);
  if (status < 0) return status;

  HIPCHK(hipEventRecord(g->ev1, g->stream));
  HIPCHK(hipEventSynchronize(g->ev1));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
  if (st) {
    st->status = status;
    st->iters = ks.iters;
    st->restarts = ks.restarts;
    st->rel_res = ks.rel;
    st->rel_res_true = ks.rel_true;
    st->ms = ms;
    st->floor_est = ks.floor_est;
  }
  return status;
}

void default_opts(int32_t op, bf_solver_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->ksp = BF_KSP_CG;
  o->pc = BF_PC_MG;
  o->maxit = 200;
  o->restart = 30;
  o->smoother = BF_SMOOTH_CHEBYSHEV;
  o->degree = 0;
  o->check_every = 1;
  o->max_restarts = 3;
  o->rtol = 1e-10;
  o->ratio = 0.0;
  o->omega = 0.0;
  o->mg_precision = BF_MG_F64;
  (void)op;
}

int check_grid(const bf_grid* g) {
  if (!g) return fail(BF_EINVAL, "null grid");
  return BF_OK;
}

// Parameters of a time step, checked before the step writes anything: a step
// that returns BF_EINVAL leaves the caller's fields as they were.
int check_params(const bf_params* prm) {
  if (!prm) return fail(BF_EINVAL, "null parameters");
  if (!(prm->dt > 0) || !std::isfinite(prm->dt)) return fail(BF_EINVAL, "dt must be finite and > 0");
  if (!(prm->M >= 0) || !std::isfinite(prm->M)) return fail(BF_EINVAL, "M must be finite and >= 0");
  if (!(prm->kappa >= 0) || !std::isfinite(prm->kappa))
    return fail(BF_EINVAL, "kappa must be finite and >= 0");
  if (!(prm->Npoly > 0) || !std::isfinite(prm->Npoly) || !std::isfinite(prm->chi))
    return fail(BF_EINVAL, "Npoly must be finite and > 0, chi finite");
  if (!(prm->phi_lo > 0 && prm->phi_lo < prm->phi_hi && prm->phi_hi < 1))
    return fail(BF_EINVAL, "need 0 < phi_lo < phi_hi < 1");
  const double c = prm->dt * prm->M * prm->kappa;
  if (!std::isfinite(c)) return fail(BF_EINVAL, "dt*M*kappa must be finite");
  return BF_OK;
}

// The options a solve of operator op will use (o, or the defaults when o is
// NULL), checked up front.
int resolve_opts(int op, const bf_solver_opts* o, bf_solver_opts* out) {
  if (o) {
    *out = *o;
  } else {
    default_opts(op, out);
  }
  return check_opts(*out);
}

}  // namespace

// ------------------------------------------------ allocation-free scratch
// Device memory of the allocation-free entry point (bf_residual_noalloc):
// two groups of reduction partials (at most kStreamMaxBlocks each: a tiled
// reduction launches at most that many workgroups, the one-thread-per-node
// form red_blocks(n) <= kMaxRedBlocks) and the scalar slots their finalize
// kernels write.  264 KB per GPU, held until the process ends; every call on
// a GPU shares that GPU's copy, so calls that overlap on one GPU race.
namespace {
constexpr int kScratchParts = kStreamMaxBlocks;
constexpr int kScratchSlots = 16;
static_assert(kMaxRedBlocks <= kScratchParts, "partials of the untiled reductions");
static_assert(S_ULP2 < kScratchSlots && S_RTRUE < kScratchSlots && S_BN2 < kScratchSlots,
              "scalar slots of the residual norms");
constexpr int kScratchDevices = 64;
constexpr int kNoallocMaxN = 32768;  // the largest grid the library accepts

static __device__ __align__(256) double scratch[2 * kScratchParts + kScratchSlots];

std::mutex g_scratch_mu;
double* g_scratch_dev[kScratchDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy at its own address; in host code the
// array's name is only a stand-in and must not be passed to a kernel).
int scratch_on_current_device(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices)
    return fail(BF_EUNSUPPORTED, "device %d: the scratch table covers devices 0..%d", dev,
                kScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(BF_EHIP, "hipGetSymbolAddress returned a null address");
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return BF_OK;
}
}  // namespace

// Host helpers shared with the ensemble driver (host.hpp).
namespace bf {
int host_fail(int code, const char* msg) { return fail(code, "%s", msg); }
OpDesc host_level_op(int op, int n, double c) { return level_op(op, n, c); }
int host_smoother(int op, int n, double c, const bf_solver_opts& o, double* a, double* g) {
  const Smoother S = make_smoother(op, n, c, o);
  for (int k = 0; k < 8; ++k) {
    a[k] = S.a[k];
    g[k] = S.g[k];
  }
  return S.degree;
}
int host_coarse_operator(int op, double c, std::vector<double>& G) {
  return coarse_operator(op, c, G);
}
double host_column_sq(const OpDesc& A) { return column_sq(A); }
void host_default_opts(int op, bf_solver_opts* o) { default_opts(op, o); }
int host_check_opts(const bf_solver_opts& o) { return check_opts(o); }
}  // namespace bf

// ====================================================================== C ABI
extern "C" {

void bf_solver_opts_default(int32_t op, bf_solver_opts* o) {
  if (o) default_opts(op, o);
}

const char* bf_last_error(void) { return g_err.c_str(); }

int bf_grid_create(const bf_grid_desc* desc, bf_grid** out) {
  g_err.clear();
  if (!desc || !out) return fail(BF_EINVAL, "null argument");
  *out = nullptr;
  const int n = desc->n;
  if (!is_pow2(n) || n < kCoarseN || n > 32768)
    return fail(BF_EINVAL, "n = %d must be a power of two in [4, 32768]", n);
  if (desc->dtype != BF_F64) return fail(BF_EUNSUPPORTED, "dtype %d not supported", desc->dtype);
  bf_grid* g = new bf_grid();
  g->n = n;
  g->npts = (int64_t)(n + 1) * n;
  g->stream = (hipStream_t)desc->stream;
  int s = BF_OK;
  auto A = [&](double** p, int64_t cnt) {
    if (s == BF_OK) s = dalloc(g, p, cnt);
  };
  for (int m = n; m >= kCoarseN; m /= 2) {
    Level L;
    L.n = m;
    L.npts = (int64_t)(m + 1) * m;
    A(&L.xa, L.npts);
    A(&L.xb, L.npts);
    A(&L.r, L.npts);
    A(&L.b, L.npts);
    g->lv.push_back(L);
  }
  A(&g->r, g->npts);
  A(&g->z, g->npts);
  A(&g->p, g->npts);
  A(&g->p2, g->npts);
  A(&g->q, g->npts);
  A(&g->work_b, g->npts);
  A(&g->work_p, g->npts);
  A(&g->work_mu, g->npts);
  A(&g->scal, kNumSlots);
  A(&g->partials, (int64_t)kMaxRedBlocks * 72);
  A(&g->coarse_ch, kCoarseSize * kCoarseSize);
  A(&g->coarse_lap, kCoarseSize * kCoarseSize);
  A(&g->coarse_helm, kCoarseSize * kCoarseSize);
  if (s == BF_OK) {
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(int32_t) * 4) != hipSuccess)
      s = fail(BF_ENOMEM, "counter allocation failed");
    else {
      g->counter = (int32_t*)p;
      g->allocs.push_back(p);
    }
  }
  if (s == BF_OK && hipHostMalloc((void**)&g->h_scal, sizeof(double) * kNumSlots) != hipSuccess)
    s = fail(BF_ENOMEM, "pinned host allocation failed");
  if (s == BF_OK) std::memset(g->h_scal, 0, sizeof(double) * kNumSlots);
  if (s == BF_OK && (hipEventCreate(&g->ev0) != hipSuccess || hipEventCreate(&g->ev1) != hipSuccess))
    s = fail(BF_EHIP, "event creation failed");
  if (s == BF_OK && hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking) != hipSuccess)
    s = fail(BF_EHIP, "capture stream creation failed");
  {
    const char* nr = std::getenv("BF_NO_RING");
    if (nr && nr[0] == '1') g->ring_m = 0;  // the CG step updates x itself
    const char* fb = std::getenv("BF_FLEX_BETA");
    if (fb && fb[0] == '1') g->flex_beta = true;
    const char* ng = std::getenv("BF_NO_GRAPHS");
    if (ng && ng[0] == '1') g->use_graphs = false;
    // V-cycles are replayed from captured graphs on grids up to 2048^2
    // (BF_GRAPH_MAX_N).  Above, the kernels of a V-cycle take far longer than
    // the host needs to launch them, and the eager sequence avoids the gaps at
    // a graph's entry and exit (about 5 and 8 us): 4096^2 mixed step 11.51
    // against 11.58 ms with graphs.
    const char* gm = std::getenv("BF_GRAPH_MAX_N");
    if (g->n > (gm ? std::atoi(gm) : 2048)) g->use_graphs = false;
    const char* no = std::getenv("BF_NO_OVERLAP");
    if (no && no[0] == '1') g->overlap = false;
  }
  if (s == BF_OK) {
    launch_fill(kNumSlots, g->scal, 0.0, g->stream);
    launch_fill(g->npts, g->q, 0.0, g->stream);
    s = upload_coarse(g, BF_OP_LAP, 0.0);
  }
  if (s != BF_OK) {
    std::string keep = g_err;
    bf_grid_destroy(g);
    g_err = keep;
    return s;
  }
  *out = g;
  return BF_OK;
}

int bf_grid_destroy(bf_grid* g) {
  if (!g) return BF_OK;
  if (g->twin) bf_grid_destroy(g->twin);
  if (g->twin_stream) (void)hipStreamDestroy(g->twin_stream);
  if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
  if (g->ev_join) (void)hipEventDestroy(g->ev_join);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  else (void)hipDeviceSynchronize();
  for (auto& e : g->graphs) (void)hipGraphExecDestroy(e.exec);
  g->graphs.clear();
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  for (void* p : g->allocs)
    if (p) (void)hipFree(p);
  if (g->h_scal) (void)hipHostFree(g->h_scal);
  if (g->ev0) (void)hipEventDestroy(g->ev0);
  if (g->ev1) (void)hipEventDestroy(g->ev1);
  for (hipEvent_t e : g->cg_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : g->ru_ev) (void)hipEventDestroy(e);
  delete g;
  return BF_OK;
}

int bf_grid_cg_timing(bf_grid* g, int32_t enable) {
  TRY(check_grid(g));
  if (enable < 0) return fail(BF_EINVAL, "timing period %d must be >= 0", (int)enable);
  g->cg_timing = enable;
  if (g->cg_timing) {
    g->cg_used = 0;
    g->ru_used = 0;
    g->cg_count = 0;
    g->cg_first.clear();
  }
  return BF_OK;
}

int bf_grid_cg_timing_read(bf_grid* g, double* total_ms, int64_t* launches,
                           int64_t* first_launches) {
  TRY(check_grid(g));
  HIPCHK(hipStreamSynchronize(g->stream));
  double tot = 0.0;
  int64_t nf = 0;
  for (size_t k = 0; k + 1 < g->cg_used; k += 2) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, g->cg_ev[k], g->cg_ev[k + 1]));
    tot += ms;
  }
  for (uint8_t f : g->cg_first) nf += f;
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)g->cg_first.size();
  if (first_launches) *first_launches = nf;
  g->cg_used = 0;
  g->cg_first.clear();
  return BF_OK;
}

int bf_grid_rupdate_timing_read(bf_grid* g, double* total_ms, int64_t* launches) {
  TRY(check_grid(g));
  HIPCHK(hipStreamSynchronize(g->stream));
  double tot = 0.0;
  for (size_t k = 0; k + 1 < g->ru_used; k += 2) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, g->ru_ev[k], g->ru_ev[k + 1]));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)(g->ru_used / 2);
  g->ru_used = 0;
  return BF_OK;
}

int bf_grid_shape(const bf_grid* g, int64_t* rows, int64_t* cols) {
  TRY(check_grid(g));
  if (rows) *rows = g->n + 1;
  if (cols) *cols = g->n;
  return BF_OK;
}

int bf_apply(bf_grid* g, int32_t op, double c, const double* x, double* y) {
  TRY(check_grid(g));
  if (!x || !y) return fail(BF_EINVAL, "null field");
  if (x == y) return fail(BF_EINVAL, "x and y must not alias");
  if (op != BF_OP_LAP && op != BF_OP_CH && op != BF_OP_HELM) return fail(BF_EINVAL, "op %d", op);
  launch_apply(level_op(op, g->n, c), x, y, g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_solve_ch(bf_grid* g, double c, const double* b, double* x, const bf_solver_opts* o,
                bf_solve_stats* st) {
  TRY(check_grid(g));
  if (!b || !x) return fail(BF_EINVAL, "null field");
  if (b == x) return fail(BF_EINVAL, "b and x must not alias");
  if (!(c >= 0) || !std::isfinite(c)) return fail(BF_EINVAL, "c = %g must be finite and >= 0", c);
  bf_solver_opts d;
  default_opts(BF_OP_CH, &d);
  const int s = run_krylov(g, BF_OP_CH, c, b, x, o ? *o : d, st);
  return s;
}

int bf_solve_pressure(bf_grid* g, const double* rhs, double* p, const bf_solver_opts* o,
                      bf_solve_stats* st) {
  TRY(check_grid(g));
  if (!rhs || !p) return fail(BF_EINVAL, "null field");
  if (rhs == p) return fail(BF_EINVAL, "rhs and p must not alias");
  bf_solver_opts d;
  default_opts(BF_OP_LAP, &d);
  const bf_solver_opts& oo = o ? *o : d;
  TRY(check_opts(oo));
  // projected copy of the right-hand side (null space of constants)
  wdot_async(g, rhs, nullptr, F_MEAN, 0);
  launch_sub_mean(g->n, rhs, g->work_p, g->scal, g->stream);
  const int s = run_krylov(g, BF_OP_LAP, 0.0, g->work_p, p, oo, st);
  if (s < 0) return s;
  wdot_async(g, p, nullptr, F_MEAN, 0);
  launch_sub_mean(g->n, p, p, g->scal, g->stream);
  HIPCHK(hipStreamSynchronize(g->stream));
  return s;
}

int bf_ch_rhs(bf_grid* g, const bf_params* prm, const double* phi, double* b, int32_t* clamped) {
  TRY(check_grid(g));
  if (!prm || !phi || !b) return fail(BF_EINVAL, "null argument");
  if (phi == b) return fail(BF_EINVAL, "phi and b must not alias");
  if (!(prm->Npoly > 0) || !(prm->phi_lo > 0) || !(prm->phi_hi < 1) || !(prm->phi_lo < prm->phi_hi))
    return fail(BF_EINVAL, "bad Flory-Huggins parameters");
  if (clamped) launch_fill_i32(1, clamped, 0, g->stream);
  launch_ch_rhs(g->n, phi, nullptr, phi, b, g->work_mu, prm->dt * prm->M, 1.0 / prm->Npoly,
                prm->chi, prm->phi_lo, prm->phi_hi, clamped, g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_pressure_rhs(bf_grid* g, double dt, const double* u, const double* v, double* rhs) {
  TRY(check_grid(g));
  if (!u || !v || !rhs) return fail(BF_EINVAL, "null field");
  if (!(dt > 0)) return fail(BF_EINVAL, "dt must be > 0");
  if (rhs == u || rhs == v) return fail(BF_EINVAL, "rhs must not alias u or v");
  launch_divergence(g->n, u, v, rhs, (double)g->n / (2.0 * dt), g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_velocity_correct(bf_grid* g, double dt, const double* p, const double* ustar,
                        const double* vstar, double* u, double* v) {
  TRY(check_grid(g));
  if (!p || !ustar || !vstar) return fail(BF_EINVAL, "null field");
  if (p == u || p == v) return fail(BF_EINVAL, "p must not alias u or v");
  launch_velocity(g->n, p, ustar, vstar, u, v, dt * (double)g->n * 0.5, g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

namespace {

// bf_solve_pressure from p = 0 (the pressure solve of a time step): one pass
// projects the right-hand side into b, writes it as the initial residual
// (r = b - A 0 = b; in float32 too for the float32 V-cycle) and reduces
// ||b||_W^2, so CG starts without a residual pass and a norm pass of its own.
int solve_pressure_zero(bf_grid* g, const double* rhs, double* p, const bf_solver_opts* o,
                        bf_solve_stats* st) {
  if (rhs == p) return fail(BF_EINVAL, "rhs and p must not alias");
  bf_solver_opts d;
  default_opts(BF_OP_LAP, &d);
  const bf_solver_opts& oo = o ? *o : d;
  TRY(check_opts(oo));
  const bool mixed = oo.pc == BF_PC_MG && oo.mg_precision == BF_MG_F32;
  if (mixed) TRY(ensure_mixed(g));
  const int np = nparts_of(g);
  wdot_async(g, rhs, nullptr, F_MEAN, 0);
  launch_project_start(g->n, rhs, g->work_p, g->r, mixed ? g->r32 : nullptr, g->scal,
                       g->partials, np, g->stream);
  launch_finalize(g->partials, np, g->scal, F_STORE, S_BN2, g->n, g->stream);
  launch_fill(g->npts, p, 0.0, g->stream);
  TRY(read_scalars(g, S_BN2 + 1));
  g->bn2_b = g->work_p;
  g->r_is_b = oo.ksp == BF_KSP_CG;
  const int s = run_krylov(g, BF_OP_LAP, 0.0, g->work_p, p, oo, st);
  if (s < 0) return s;
  wdot_async(g, p, nullptr, F_MEAN, 0);
  launch_sub_mean(g->n, p, p, g->scal, g->stream);
  HIPCHK(hipStreamSynchronize(g->stream));
  return s;
}

// The pressure half of a step on grid h (its stream, its workspaces).
int pressure_half(bf_grid* h, const bf_params* prm, const double* ustar, const double* vstar,
                  double* p, double* u, double* v, const bf_solver_opts* pr, bf_solve_stats* S) {
  TRY(bf_pressure_rhs(h, prm->dt, ustar, vstar, h->work_b));
  const int s = solve_pressure_zero(h, h->work_b, p, pr, S);
  if (s < 0) return s;
  if (u || v) TRY(bf_velocity_correct(h, prm->dt, p, ustar, vstar, u, v));
  return s;
}

int scale_guess(bf_grid* g, const double* b, double* x);
int apply_guess(bf_grid* g, double* x);

// Initial guess of the Cahn-Hilliard solve of a time step (x holds phi^n on
// entry): x0 = gamma phi^n with gamma minimising ||b - gamma A phi^n||_W, or 0
// when no gamma beats the zero guess (<b, A phi^n>_W <= 0).  Once phi is
// smooth, phi^n is close to phi^{n+1}: at 4096^2 its relative residual is
// 3e-2 ... 8e-3 from the third step on (against 1 for the zero guess), about
// three CG iterations fewer; on the first steps from the noisy initial state
// c L^2 phi^n is huge (relative residual 3e5, then 50) and gamma is tiny.
int ch_guess(bf_grid* g, double c, const double* b, double* x) {
  const OpDesc A = level_op(BF_OP_CH, g->n, c);
  g->bn2_b = nullptr;
  g->r_is_b = false;
  if (stream_ok(g->n)) {
    // <b, A x>, <A x, A x> and ||b||^2 in one pass (A x is not stored)
    hipStream_t st = g->stream;
    const int np = stream_guess(A, x, b, g->partials, st);
    launch_finalize(g->partials, np, g->scal, F_STORE, S_GB, g->n, st);
    launch_finalize(g->partials + np, np, g->scal, F_STORE, S_GG, g->n, st);
    launch_finalize(g->partials + 2 * np, np, g->scal, F_STORE, S_BN2, g->n, st);
    TRY(read_scalars(g, S_GG + 1));
    g->bn2_b = b;
    return apply_guess(g, x);
  }
  launch_apply(A, x, g->q, g->stream);  // q = A phi^n (float64: only gamma depends on it)
  return scale_guess(g, b, x);
}

// The common part of the least-squares initial guesses: with q = A x in g->q,
// x = gamma x, gamma = <b, q>_W / <q, q>_W, or x = 0 when gamma would not be
// positive.
int scale_guess(bf_grid* g, const double* b, double* x) {
  wdot_async(g, b, g->q, F_STORE, S_GB);
  wdot_async(g, g->q, g->q, F_STORE, S_GG);
  TRY(read_scalars(g, S_GG + 1));
  return apply_guess(g, x);
}

// x = gamma x with gamma = <b, q>_W / <q, q>_W from h_scal[S_GB], h_scal[S_GG],
// or x = 0 when gamma would not be positive.
int apply_guess(bf_grid* g, double* x) {
  hipStream_t st = g->stream;
  const double bq = g->h_scal[S_GB], qq = g->h_scal[S_GG];
  if (!std::isfinite(bq) || !std::isfinite(qq)) return fail(BF_ENONFINITE, "phi is not finite");
  if (!(bq > 0.0 && qq > 0.0)) {
    launch_fill(g->npts, x, 0.0, st);
    return BF_OK;
  }
  g->h_scal[S_GAMMA] = bq / qq;
  HIPCHK(hipMemcpyAsync(g->scal + S_GAMMA, g->h_scal + S_GAMMA, sizeof(double),
                        hipMemcpyHostToDevice, st));
  launch_scale(g->n, x, x, g->scal, S_GAMMA, 0, st);
  return BF_OK;
}

int ensure_twin(bf_grid* g) {
  if (g->twin) return BF_OK;
  HIPCHK(hipStreamCreateWithFlags(&g->twin_stream, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming));
  bf_grid_desc d;
  d.n = g->n;
  d.dtype = BF_F64;
  d.stream = g->twin_stream;
  return bf_grid_create(&d, &g->twin);
}

}  // namespace

int bf_step(bf_grid* g, const bf_params* prm, double* phi, const double* ustar,
            const double* vstar, double* p, double* u, double* v, const bf_solver_opts* ch,
            const bf_solver_opts* pr, bf_solve_stats stats[2]) {
  TRY(check_grid(g));
  if (!prm || !phi || !ustar || !vstar || !p) return fail(BF_EINVAL, "null argument");
  if (phi == p || phi == ustar || phi == vstar || (u && u == phi) || (v && v == phi))
    return fail(BF_EINVAL, "phi must not alias p, u*, v*, u or v");
  // everything either half could reject is checked before phi or p is written
  TRY(check_params(prm));
  bf_solver_opts och, opr;
  TRY(resolve_opts(BF_OP_CH, ch, &och));
  TRY(resolve_opts(BF_OP_LAP, pr, &opr));
  ch = &och;
  pr = &opr;
  bf_solve_stats local[2];
  bf_solve_stats* S = stats ? stats : local;
  std::memset(S, 0, sizeof(bf_solve_stats) * 2);
  if (g->overlap && ensure_twin(g) == BF_OK) {
    // fork: the pressure half waits for the caller's prior work on its own stream
    HIPCHK(hipEventRecord(g->ev_fork, g->stream));
    HIPCHK(hipStreamWaitEvent(g->twin_stream, g->ev_fork, 0));
    int s2 = BF_OK;
    std::string err2;
    std::thread th([&] {
      s2 = pressure_half(g->twin, prm, ustar, vstar, p, u, v, pr, &S[1]);
      if (s2 < 0) err2 = bf_last_error();
    });
    const double c = prm->dt * prm->M * prm->kappa;
    int s1 = bf_ch_rhs(g, prm, phi, g->work_b, g->counter);
    if (s1 >= 0) s1 = ch_guess(g, c, g->work_b, phi);
    if (s1 >= 0) s1 = bf_solve_ch(g, c, g->work_b, phi, ch, &S[0]);
    th.join();
    HIPCHK(hipEventRecord(g->ev_join, g->twin_stream));
    HIPCHK(hipStreamWaitEvent(g->stream, g->ev_join, 0));
    if (s1 < 0) return s1;
    if (s2 < 0) return fail(s2, "%s", err2.c_str());
    int32_t clamped = 0;
    HIPCHK(hipMemcpyAsync(&clamped, g->counter, sizeof(int32_t), hipMemcpyDeviceToHost,
                          g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    S[0].clamped = clamped;
    return s1 > s2 ? s1 : s2;
  }
  (void)hipGetLastError();
  TRY(bf_ch_rhs(g, prm, phi, g->work_b, g->counter));
  const double c = prm->dt * prm->M * prm->kappa;
  TRY(ch_guess(g, c, g->work_b, phi));
  const int s1 = bf_solve_ch(g, c, g->work_b, phi, ch, &S[0]);
  if (s1 < 0) return s1;
  TRY(bf_pressure_rhs(g, prm->dt, ustar, vstar, g->work_b));
  const int s2 = solve_pressure_zero(g, g->work_b, p, pr, &S[1]);
  if (s2 < 0) return s2;
  if (u || v) TRY(bf_velocity_correct(g, prm->dt, p, ustar, vstar, u, v));
  int32_t clamped = 0;
  HIPCHK(hipMemcpyAsync(&clamped, g->counter, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  S[0].clamped = clamped;
  return s1 > s2 ? s1 : s2;
}

int bf_solve_helmholtz(bf_grid* g, double beta, const double* b, double* x,
                       const bf_solver_opts* o, bf_solve_stats* st) {
  TRY(check_grid(g));
  if (!b || !x) return fail(BF_EINVAL, "null field");
  if (b == x) return fail(BF_EINVAL, "b and x must not alias");
  if (!(beta >= 0) || !std::isfinite(beta))
    return fail(BF_EINVAL, "beta = %g must be finite and >= 0", beta);
  bf_solver_opts d;
  default_opts(BF_OP_HELM, &d);
  return run_krylov(g, BF_OP_HELM, beta, b, x, o ? *o : d, st);
}

int bf_apply_mob(bf_grid* g, double c, const double* m, const double* x, double* y) {
  TRY(check_grid(g));
  if (!m || !x || !y) return fail(BF_EINVAL, "null field");
  if (y == x || y == m) return fail(BF_EINVAL, "y must not alias x or m");
  if (!(c >= 0) || !std::isfinite(c)) return fail(BF_EINVAL, "c = %g must be finite and >= 0", c);
  launch_mob(g->n, c, m, x, nullptr, y, nullptr, 0, g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_solve_ch_mob(bf_grid* g, double c, const double* m, const double* b, double* x,
                    const bf_solver_opts* o, bf_solve_stats* st) {
  TRY(check_grid(g));
  if (!m || !b || !x) return fail(BF_EINVAL, "null field");
  if (b == x || m == x) return fail(BF_EINVAL, "x must not alias b or m");
  if (!(c >= 0) || !std::isfinite(c)) return fail(BF_EINVAL, "c = %g must be finite and >= 0", c);
  bf_solver_opts d;
  default_opts(BF_OP_CH, &d);
  d.ksp = BF_KSP_GMRES;
  d.restart = 10;  // at 4096^2: 231 ms per step against 320 with GMRES(30) (orthogonalisation)
  const bf_solver_opts& oo = o ? *o : d;
  // the preconditioner: the constant-mobility operator at the weighted mean
  // mobility, rounded to 6 significant bits so that steps whose mean differs
  // only by rounding (the mass is conserved) reuse one captured V-cycle
  wdot_async(g, m, nullptr, F_MEAN, 0);
  TRY(read_scalars(g, S_MEAN + 1));
  const double mm = g->h_scal[S_MEAN];
  if (!(mm > 0) || !std::isfinite(mm))
    return fail(BF_EINVAL, "the mobility must have a positive, finite mean");
  int e2 = 0;
  const double fr = std::frexp(mm, &e2);
  g->mob = m;
  g->mob_pre = std::ldexp(std::round(std::ldexp(fr, 6)), e2 - 6);
  if (oo.pc == BF_PC_MG) {
    if (oo.mg_precision == BF_MG_F32) {
      TRY(ensure_mixed(g));
      TRY(setup_mob_levels<float>(g, g->lvf, m));
    } else {
      TRY(setup_mob_levels<double>(g, g->lv, m));
    }
  }
  const int s = run_krylov(g, kOpMob, c, b, x, oo, st);
  g->mob = nullptr;
  return s;
}

int bf_step_ch_mob(bf_grid* g, const bf_params* prm, double* phi, const bf_solver_opts* o,
                   bf_solve_stats* stats) {
  TRY(check_grid(g));
  if (!prm || !phi) return fail(BF_EINVAL, "null argument");
  TRY(check_params(prm));
  if (!(prm->M > 0)) return fail(BF_EINVAL, "M must be > 0 (the mobility is M clamp(phi))");
  if (o) {
    bf_solver_opts oo;
    TRY(resolve_opts(BF_OP_CH, o, &oo));
    if (oo.ksp != BF_KSP_GMRES)
      return fail(BF_EINVAL, "the variable-mobility operator is not symmetric: use GMRES");
  }
  if (!g->work_m) TRY(dalloc(g, &g->work_m, g->npts));
  hipStream_t st = g->stream;
  launch_fill_i32(1, g->counter, 0, st);
  launch_mob_rhs(g->n, phi, g->work_m, g->work_mu, g->work_b, prm->M, prm->dt, 1.0 / prm->Npoly,
                 prm->chi, prm->phi_lo, prm->phi_hi, g->counter, st);
  // start from gamma phi^n, the least-squares multiple for the mobility operator
  launch_mob(g->n, prm->dt * prm->kappa, g->work_m, phi, nullptr, g->q, nullptr, 0, st);
  HIPCHK(hipGetLastError());
  TRY(scale_guess(g, g->work_b, phi));
  bf_solve_stats local;
  bf_solve_stats* S = stats ? stats : &local;
  std::memset(S, 0, sizeof(*S));
  const int s = bf_solve_ch_mob(g, prm->dt * prm->kappa, g->work_m, g->work_b, phi, o, S);
  if (s < 0) return s;
  int32_t clamped = 0;
  HIPCHK(hipMemcpyAsync(&clamped, g->counter, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  S->clamped = clamped;
  return s;
}

int bf_momentum_predict(bf_grid* g, double dt, double nu, double theta, double U,
                        const double* u, const double* v, double* ustar, double* vstar,
                        const bf_solver_opts* o, bf_solve_stats stats[2]) {
  TRY(check_grid(g));
  if (!u || !v || !ustar || !vstar) return fail(BF_EINVAL, "null field");
  if (ustar == vstar || u == vstar || v == ustar || u == v)
    return fail(BF_EINVAL, "the two components must not alias each other");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(BF_EINVAL, "dt must be finite and > 0");
  if (!(nu >= 0) || !std::isfinite(nu)) return fail(BF_EINVAL, "nu must be finite and >= 0");
  if (!(theta >= 0 && theta <= 1)) return fail(BF_EINVAL, "theta must lie in [0, 1]");
  if (!std::isfinite(U)) return fail(BF_EINVAL, "U must be finite");
  bf_solver_opts d;
  default_opts(BF_OP_HELM, &d);
  const bf_solver_opts& oo = o ? *o : d;
  TRY(check_opts(oo));
  bf_solve_stats local[2];
  bf_solve_stats* S = stats ? stats : local;
  std::memset(S, 0, sizeof(bf_solve_stats) * 2);
  const double beta = theta * dt * nu;
  // both right-hand sides first (they read u and v), then the initial guesses
  launch_momentum_rhs(g->n, u, v, dt, (1.0 - theta) * dt * nu, U, g->work_b, g->work_mu,
                      g->stream);
  if (ustar != u) launch_copy(g->npts, u, ustar, g->stream);
  if (vstar != v) launch_copy(g->npts, v, vstar, g->stream);
  HIPCHK(hipGetLastError());
  if (g->overlap && ensure_twin(g) == BF_OK) {
    // the two component solves are independent: the y component runs on the twin grid
    HIPCHK(hipEventRecord(g->ev_fork, g->stream));
    HIPCHK(hipStreamWaitEvent(g->twin_stream, g->ev_fork, 0));
    int s2 = BF_OK;
    std::string err2;
    std::thread th([&] {
      s2 = bf_solve_helmholtz(g->twin, beta, g->work_mu, vstar, &oo, &S[1]);
      if (s2 < 0) err2 = bf_last_error();
    });
    const int s1 = bf_solve_helmholtz(g, beta, g->work_b, ustar, &oo, &S[0]);
    th.join();
    HIPCHK(hipEventRecord(g->ev_join, g->twin_stream));
    HIPCHK(hipStreamWaitEvent(g->stream, g->ev_join, 0));
    if (s1 < 0) return s1;
    if (s2 < 0) return fail(s2, "%s", err2.c_str());
    return s1 > s2 ? s1 : s2;
  }
  (void)hipGetLastError();
  const int s1 = bf_solve_helmholtz(g, beta, g->work_b, ustar, &oo, &S[0]);
  if (s1 < 0) return s1;
  const int s2 = bf_solve_helmholtz(g, beta, g->work_mu, vstar, &oo, &S[1]);
  if (s2 < 0) return s2;
  return s1 > s2 ? s1 : s2;
}

int bf_step_ch(bf_grid* g, const bf_params* prm, double* phi, const double* u, const double* v,
               const bf_solver_opts* o, bf_solve_stats* stats) {
  TRY(check_grid(g));
  if (!prm || !phi) return fail(BF_EINVAL, "null argument");
  if ((u == nullptr) != (v == nullptr)) return fail(BF_EINVAL, "u and v must both be given or both be null");
  if (u && (u == phi || v == phi)) return fail(BF_EINVAL, "u, v must not alias phi");
  TRY(check_params(prm));
  bf_solver_opts oo;
  TRY(resolve_opts(BF_OP_CH, o, &oo));
  o = &oo;
  bf_solve_stats local;
  bf_solve_stats* S = stats ? stats : &local;
  std::memset(S, 0, sizeof(*S));
  TRY(bf_ch_rhs(g, prm, phi, g->work_b, g->counter));
  if (u) launch_advect_sub(g->n, phi, u, v, g->work_b, prm->dt, g->stream);
  const double c = prm->dt * prm->M * prm->kappa;
  TRY(ch_guess(g, c, g->work_b, phi));
  const int s = bf_solve_ch(g, c, g->work_b, phi, o, S);
  if (s < 0) return s;
  int32_t clamped = 0;
  HIPCHK(hipMemcpyAsync(&clamped, g->counter, sizeof(int32_t), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  S->clamped = clamped;
  return s;
}

int bf_step_ch_cn(bf_grid* g, const bf_params* prm, double* phi, double* phi_prev, int32_t first,
                  const bf_solver_opts* o, bf_solve_stats* stats) {
  TRY(check_grid(g));
  if (!prm || !phi || !phi_prev) return fail(BF_EINVAL, "null argument");
  if (phi == phi_prev) return fail(BF_EINVAL, "phi and phi_prev must not alias");
  // checked before phi_prev receives phi^n or phi the initial guess
  TRY(check_params(prm));
  bf_solver_opts oo;
  TRY(resolve_opts(BF_OP_CH, o, &oo));
  o = &oo;
  const double c = prm->dt * prm->M * prm->kappa;
  bf_solve_stats local;
  bf_solve_stats* S = stats ? stats : &local;
  std::memset(S, 0, sizeof(*S));
  hipStream_t st = g->stream;
  // b = (I - c/2 L^2) phi^n + dt M L mu(phi*); the explicit operator is
  // applied with the double-double stencil sum: in plain float64 its
  // rounding (about u * 32 c n^4 |phi|) would reach 1e-10 of phi at 1024^2
  launch_apply_dot(level_op(BF_OP_CH, g->n, -0.5 * c), phi, g->work_b, g->partials,
                   nparts_of(g), st, true);
  launch_fill_i32(1, g->counter, 0, st);
  launch_ch_rhs(g->n, phi, first ? nullptr : phi_prev, g->work_b, g->work_b, g->work_mu,
                prm->dt * prm->M, 1.0 / prm->Npoly, prm->chi, prm->phi_lo, prm->phi_hi,
                g->counter, st);
  launch_copy(g->npts, phi, phi_prev, st);
  TRY(ch_guess(g, 0.5 * c, g->work_b, phi));
  const int s = bf_solve_ch(g, 0.5 * c, g->work_b, phi, o, S);
  if (s < 0) return s;
  int32_t clamped = 0;
  HIPCHK(hipMemcpyAsync(&clamped, g->counter, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  S->clamped = clamped;
  return s;
}

int bf_adjoint_step(bf_grid* g, const bf_params* prm, const double* phi_n, const double* u,
                    const double* v, const double* du, const double* dv,
                    const double* lambda_in, double* lambda_out, double grads[2],
                    const bf_solver_opts* o, bf_solve_stats* stats) {
  TRY(check_grid(g));
  if (!prm || !phi_n || !lambda_in || !lambda_out) return fail(BF_EINVAL, "null argument");
  if ((u == nullptr) != (v == nullptr)) return fail(BF_EINVAL, "u and v must both be given or both be null");
  if ((du == nullptr) != (dv == nullptr)) return fail(BF_EINVAL, "du and dv must both be given or both be null");
  if (lambda_out == phi_n || (u && (lambda_out == u || lambda_out == v)) ||
      (du && (lambda_out == du || lambda_out == dv)))
    return fail(BF_EINVAL, "lambda_out must not alias phi_n, u, v, du or dv");
  TRY(check_params(prm));
  bf_solver_opts oo;
  TRY(resolve_opts(BF_OP_CH, o, &oo));
  o = &oo;
  if (!g->work_e) TRY(dalloc(g, &g->work_e, g->npts));
  hipStream_t st = g->stream;
  // eta = A^{-T} lam = W A^{-1} W^{-1} lam: solve A e = W^{-1} lam, eta = W e
  launch_wscale(g->n, lambda_in, g->work_b, true, st);
  launch_fill(g->npts, g->work_e, 0.0, st);
  const double dtM = prm->dt * prm->M;
  const int s = bf_solve_ch(g, dtM * prm->kappa, g->work_b, g->work_e, o, stats);
  if (s < 0) return s;
  AdjCoef C;
  C.dt = prm->dt;
  C.dtM = dtM;
  C.inv_npoly = 1.0 / prm->Npoly;
  C.chi = prm->chi;
  C.lo = prm->phi_lo;
  C.hi = prm->phi_hi;
  const int np = nparts_of(g);
  launch_adjoint_rhs(g->n, g->work_e, phi_n, u, v, du, dv, lambda_out, C, g->partials, np, st);
  launch_finalize(g->partials, np, g->scal, F_STORE, S_TMP, g->n, st);
  launch_finalize(g->partials + np, np, g->scal, F_STORE, S_TMP + 1, g->n, st);
  TRY(read_scalars(g, S_TMP + 2));
  if (grads) {
    grads[0] += dtM * g->h_scal[S_TMP];
    if (du) grads[1] += -prm->dt * g->h_scal[S_TMP + 1];
  }
  return s;
}

int bf_vcycle(bf_grid* g, int32_t op, double c, const bf_solver_opts* o, const double* r,
              double* z) {
  TRY(check_grid(g));
  if (!r || !z) return fail(BF_EINVAL, "null field");
  if (op != BF_OP_LAP && op != BF_OP_CH && op != BF_OP_HELM) return fail(BF_EINVAL, "op %d", op);
  bf_solver_opts d;
  default_opts(op, &d);
  const bf_solver_opts& oo = o ? *o : d;
  TRY(check_opts(oo));
  TRY(ensure_coarse(g, op, c));
  bf_solver_opts om = oo;
  om.pc = BF_PC_MG;
  if (om.mg_precision == BF_MG_F32) TRY(ensure_mixed(g));
  double* res = precondition(g, op, c, om, r);
  launch_copy(g->npts, res, z, g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_restrict(bf_grid* g, int32_t nf, const double* fine, double* coarse) {
  TRY(check_grid(g));
  if (!fine || !coarse) return fail(BF_EINVAL, "null field");
  if (!is_pow2(nf) || nf < 8 || nf > g->n) return fail(BF_EINVAL, "nf = %d", nf);
  launch_restrict(nf, fine, coarse, g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_prolong_add(bf_grid* g, int32_t nf, const double* coarse, double* fine) {
  TRY(check_grid(g));
  if (!fine || !coarse) return fail(BF_EINVAL, "null field");
  if (!is_pow2(nf) || nf < 8 || nf > g->n) return fail(BF_EINVAL, "nf = %d", nf);
  launch_prolong_add(nf, coarse, fine, g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_residual(bf_grid* g, int32_t op, double c, const double* b, const double* x, double* r,
                int32_t accurate, double* rel_norm, double* floor_est) {
  TRY(check_grid(g));
  if (!b || !x || !r) return fail(BF_EINVAL, "null field");
  if (r == x) return fail(BF_EINVAL, "r must not alias x");
  if (op != BF_OP_LAP && op != BF_OP_CH && op != BF_OP_HELM) return fail(BF_EINVAL, "op %d", op);
  if (!(c >= 0) || !std::isfinite(c)) return fail(BF_EINVAL, "c = %g must be finite and >= 0", c);
  const OpDesc A = level_op(op, g->n, c);
  const int np = nparts_of(g);
  if (!accurate) {
    const int nr = launch_residual(A, x, b, r, g->partials, np, g->stream);
    if (rel_norm) {
      launch_finalize(g->partials, nr, g->scal, F_STORE, S_RTRUE, g->n, g->stream);
      wdot_async(g, b, b, F_STORE, S_BN2);
      TRY(read_scalars(g, S_ULP2 + 1));
      *rel_norm = std::sqrt(g->h_scal[S_RTRUE] / g->h_scal[S_BN2]);
    }
    if (floor_est) *floor_est = 0.0;
    HIPCHK(hipGetLastError());
    return BF_OK;
  }
  if (!rel_norm && !floor_est) {
    launch_residual_dd(A, x, b, r, g->partials, np, g->stream);
    HIPCHK(hipGetLastError());
    return BF_OK;
  }
  wdot_async(g, b, b, F_STORE, S_BN2);
  TRY(read_scalars(g, S_BN2 + 1));
  KrylovState ks;
  const double bn = std::sqrt(g->h_scal[S_BN2]);
  TRY(true_residual(g, A, b, x, r, bn > 0 ? bn : 1.0, ks));
  if (rel_norm) *rel_norm = ks.rel_true;
  if (floor_est) *floor_est = ks.floor_est;
  return BF_OK;
}

int bf_residual_noalloc(int32_t n, int32_t op, double c, const double* b, const double* x,
                        double* r, double* norms, void* stream) {
  if (!is_pow2(n) || n < 4 || n > kNoallocMaxN)
    return fail(BF_EINVAL, "n = %d: bf_residual_noalloc takes powers of two in [4, %d]", n,
                kNoallocMaxN);
  if (!b || !x || !r || !norms) return fail(BF_EINVAL, "null field");
  if (r == x || r == b) return fail(BF_EINVAL, "r must not alias x or b");
  if (op != BF_OP_LAP && op != BF_OP_CH && op != BF_OP_HELM) return fail(BF_EINVAL, "op %d", op);
  if (!(c >= 0) || !std::isfinite(c)) return fail(BF_EINVAL, "c = %g must be finite and >= 0", c);
  const int np = red_blocks((int64_t)(n + 1) * n);
  const int nr_expected = stream_ok(n) ? stream_cfg(n).blocks : np;
  if (nr_expected > kScratchParts || g_batch.count > 1)
    return fail(BF_EINVAL, "n = %d needs %d reduction partials, the scratch holds %d", n,
                nr_expected, kScratchParts);
  double* s = nullptr;
  TRY(scratch_on_current_device(&s));
  double* parts = s;
  double* scal = s + 2 * kScratchParts;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const OpDesc A = level_op(op, n, c);
  // ||b||_W^2, then r = b - A x (double-double) with ||r||_W^2 and sum_W ulp(x)^2;
  // every partial and slot read below is written earlier on the same stream
  launch_dot(n, b, b, parts, np, st);
  launch_finalize(parts, np, scal, F_STORE, S_BN2, n, st);
  const int nr = launch_residual_dd(A, x, b, r, parts, np, st);
  launch_finalize(parts, nr, scal, F_STORE, S_RTRUE, n, st);
  launch_finalize(parts + nr, nr, scal, F_STORE, S_ULP2, n, st);
  launch_residual_norms(scal, column_sq(A), norms, st);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_smooth(bf_grid* g, int32_t op, double c, const double* x, const double* xprev,
              const double* b, double* xout, double a, double gcoef) {
  TRY(check_grid(g));
  if (!x || !b || !xout) return fail(BF_EINVAL, "null field");
  if (xout == x || xout == b) return fail(BF_EINVAL, "xout must not alias x or b");
  if (op != BF_OP_LAP && op != BF_OP_CH && op != BF_OP_HELM) return fail(BF_EINVAL, "op %d", op);
  if (!(c >= 0) || !std::isfinite(c)) return fail(BF_EINVAL, "c = %g must be finite and >= 0", c);
  launch_smooth(level_op(op, g->n, c), x, xprev, b, xout, a, gcoef, g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_copy(bf_grid* g, const double* x, double* y) {
  TRY(check_grid(g));
  if (!x || !y) return fail(BF_EINVAL, "null field");
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15)
    return fail(BF_EINVAL, "fields must be 16-byte aligned");
  launch_copy2(g->npts, x, y, g->stream);
  HIPCHK(hipGetLastError());
  return BF_OK;
}

int bf_wdot(bf_grid* g, const double* x, const double* y, double* out) {
  TRY(check_grid(g));
  if (!x || !y || !out) return fail(BF_EINVAL, "null argument");
  wdot_async(g, x, y, F_STORE, S_TMP);
  TRY(read_scalars(g, S_TMP + 1));
  *out = g->h_scal[S_TMP];
  return BF_OK;
}

}  // extern "C"
