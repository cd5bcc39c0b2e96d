// api.cpp -- C ABI entry points (include/glam.h): validation, workspace layout
// and the host control flow of the lambda path (Sec. 3, Algorithm 1; Sec. 6.4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "glam.h"
#include "launch.h"

namespace glam {

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

void set_last_error(const std::string& msg) { g_err = msg; }

Geom make_geom(const int64_t* n, const int64_t* p) {
  Geom G;
  G.n1 = (int)n[0]; G.n2 = (int)n[1]; G.n3 = (int)n[2];
  G.p1 = (int)p[0]; G.p2 = (int)p[1]; G.p3 = (int)p[2];
  G.P12 = G.p1 * G.p2;
  G.N1T = (G.n1 + 15) / 16;
  G.NJB = (G.n2 + 15) / 16;
  G.PT = (std::max(G.p1, G.p2) + 15) / 16;
  G.KB3 = (G.p3 + 15) / 16;
  G.KBN3 = (G.n3 + 15) / 16;
  G.nint = (long long)G.n3 * G.NJB * G.N1T * 256;
  G.n = (long long)G.n1 * G.n2 * G.n3;
  G.p = (long long)G.p1 * G.p2 * G.p3;
  G.t1_len = (long long)G.n3 * G.P12;
  G.s2_len = (long long)G.KBN3 * 16 * G.P12;
  G.inc_len = (long long)G.KB3 * 16 * G.P12;
  G.x3f_len = (long long)G.KB3 * 16 * G.n3;
  G.x3a_len = (long long)G.KBN3 * 16 * G.p3;
  return G;
}

static const size_t kMaxLds = 159 * 1024;   // 160 KB per CU minus static LDS

// Size checks shared by the rho-based entry points; n, p: the lifted (d = 3) sizes.
static int check_basic(int d, const int64_t* n_in, const int64_t* p_in, int dtype, int64_t* n, int64_t* p) {
  if (d != 2 && d != 3) return fail(GLAM_EINVAL, "d must be 2 or 3");
  if (!n_in || !p_in) return fail(GLAM_EINVAL, "NULL size array");
  for (int j = 0; j < d; ++j)
    if (n_in[j] < 1 || p_in[j] < 1) return fail(GLAM_EINVAL, "mode sizes must be >= 1");
  lift_sizes(d, n_in, p_in, n, p);
  for (int j = 0; j < 3; ++j) {
    if (n[j] < 1 || p[j] < 1) return fail(GLAM_EINVAL, "mode sizes must be >= 1");
    if (n[j] > (1 << 30) || p[j] > (1 << 30)) return fail(GLAM_EINVAL, "mode size too large");
  }
  if (dtype < 0 || dtype > 2) return fail(GLAM_EINVAL, "bad dtype");
  return GLAM_OK;
}

// Whether modes 1 and 2 of (n, p) in this order fit the slab kernels (why: the reason if not).
static bool inner_fit(const int64_t* n, const int64_t* p, int dtype, Geom* Gout, std::string* why) {
  if (p[0] > GLAM_MAX_INNER_P || p[1] > GLAM_MAX_INNER_P) { *why = "p_1 and p_2 must be <= GLAM_MAX_INNER_P"; return false; }
  if (n[0] > GLAM_MAX_INNER_N || n[1] > GLAM_MAX_INNER_N) { *why = "n_1 and n_2 must be <= GLAM_MAX_INNER_N"; return false; }
  Geom G = make_geom(n, p);
  if ((long long)G.n3 * G.P12 > (1LL << 40)) { *why = "problem too large"; return false; }
  if (slab_chain_lds_bytes(dtype, G) > kMaxLds) {
    *why = "modes 1-2 too large for the slab kernel's LDS budget (n_1, n_2 too big for this dtype)";
    return false;
  }
  *Gout = G;
  return true;
}

// Whether a lifted (d = 3) problem fits the slab kernels in the given order (no reordering):
// the fits decide their own mode order with it.
bool rho_order_fits(const int64_t* n, const int64_t* p, int dtype, std::string* why) {
  int64_t nl[3], pl[3];
  if (check_basic(3, n, p, dtype, nl, pl) != GLAM_OK) {
    if (why) *why = g_err;
    return false;
  }
  Geom G;
  std::string w;
  const bool ok = inner_fit(nl, pl, dtype, &G, &w);
  if (!ok && why) *why = w;
  return ok;
}

// The NLL entry points: the caller's mode order only.
static int check_sizes(int d, const int64_t* n_in, const int64_t* p_in, int dtype, Geom* Gout) {
  int64_t n[3], p[3];
  const int st = check_basic(d, n_in, p_in, dtype, n, p);
  if (st) return st;
  std::string why;
  if (!inner_fit(n, p, dtype, Gout, &why)) return fail(GLAM_EINVAL, why);
  return GLAM_OK;
}

// A rho problem and the mode order it runs in: position k holds the caller's (lifted) mode q[k].
// The caller's order when it fits the slab kernels; otherwise the fitting order with the
// largest n last (inputs and outputs are then permuted through the workspace).
struct RhoPlan {
  Geom G;                 // geometry of the order that runs
  int q[3] = {0, 1, 2};
  bool perm = false;
  bool generic = false;   // no order fits: the generic GEMM chain (rho entry points only)
  int64_t n[3], p[3];     // lifted sizes in the caller's order
};
static int plan_rho(int d, const int64_t* n_in, const int64_t* p_in, int dtype, RhoPlan* R, bool allow_generic = false) {
  int st = check_basic(d, n_in, p_in, dtype, R->n, R->p);
  if (st) return st;
  std::string why;
  if (inner_fit(R->n, R->p, dtype, &R->G, &why)) return GLAM_OK;
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 2, 0}, {1, 0, 2}, {2, 0, 1}, {2, 1, 0}};
  int best = -1;
  for (int c = 1; c < 6; ++c) {
    int64_t n[3], p[3];
    for (int k = 0; k < 3; ++k) { n[k] = R->n[perms[c][k]]; p[k] = R->p[perms[c][k]]; }
    Geom G;
    std::string w;
    if (!inner_fit(n, p, dtype, &G, &w)) continue;
    if (best < 0 || n[2] > R->n[perms[best][2]]) { best = c; R->G = G; }
  }
  if (best < 0) {
    if (allow_generic) {
      R->generic = true;
      return GLAM_OK;
    }
    return fail(GLAM_EINVAL, why + " (in every order of the modes)");
  }
  R->perm = true;
  for (int k = 0; k < 3; ++k) R->q[k] = perms[best][k];
  return GLAM_OK;
}

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of the rho / NLL entry points: k-blocked Theta, both packed copies of
// X_3, fragment-ordered T1, k-blocked S2 and per-workgroup partial sums.
struct WsLayout {
  size_t img, inc, x3f, t1, x3a, s2, part, unit, total;
};
static WsLayout ws_layout(const Geom& G, int dt) {
  const size_t es = dt_size(dt);
  WsLayout W;
  size_t o = 0;
  W.img = o; o += align256(chain_image_bytes(dt, G));
  W.inc = o; o += align256(G.inc_len * es);
  W.x3f = o; o += align256(G.x3f_len * es);
  W.t1 = o;  o += align256(G.t1_len * es);
  W.x3a = o; o += align256(G.x3a_len * es);
  W.s2 = o;  o += align256(G.s2_len * es);
  W.part = o; o += align256((size_t)G.n3 * 2 * sizeof(double));
  W.unit = o; o += 256;   // the 1 x 1 middle factor of a d = 2 model
  W.total = o;
  return W;
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free forward transform: one array per GPU, in the
// library's code object, held until the process ends.  Host code never passes the
// symbol itself to a kernel (on the host it only names a shadow); it looks up each
// device's address once, with that device current, and uses that pointer.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[GLAM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first call on that device).
static int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(GLAM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(GLAM_EDEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(GLAM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GLAM_OK;
}

#define HIPCHK(expr)                                                           \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      return fail(GLAM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    }                                                                          \
  } while (0)

}  // namespace glam

using namespace glam;

extern "C" {

const char* glam_status_string(int status) {
  switch (status) {
    case GLAM_OK: return "ok";
    case GLAM_EINVAL: return "invalid argument";
    case GLAM_ENOMEM: return "device allocation failed";
    case GLAM_EDEVICE: return "HIP runtime error";
    case GLAM_ENOCONV: return "iteration limit reached (path truncated)";
    case GLAM_ENONFINITE: return "non-finite value produced";
    default: return "unknown status";
  }
}

const char* glam_last_error(void) { return g_err.c_str(); }

const char* glam_version(void) { return "glam-mi355x 0.1.0 (gfx950)"; }

// rho workspace: the layout of the order that runs, then (reordered problems) an n-sized and
// a p-sized region of 8-byte elements for the permuted input and output
// Workspace of the generic chain: X_j^T for the forward products (dtype), two intermediates of
// general_tmp_elems elements, the unit middle factor of a d = 2 model.
struct GenWs {
  size_t xt[3], t1, t2, unit, total;
};
static GenWs gen_ws_layout(const RhoPlan& R, int dtype) {
  const size_t es = dt_size(dtype);
  GenWs W;
  size_t o = 0;
  for (int j = 0; j < 3; ++j) { W.xt[j] = o; o += align256((size_t)R.n[j] * R.p[j] * es); }
  const size_t tmp = (size_t)general_tmp_elems(R.n, R.p);
  W.t1 = o; o += align256(tmp * es);
  W.t2 = o; o += align256(tmp * es);
  W.unit = o; o += 256;
  W.total = o;
  return W;
}

static size_t rho_ws_total(const RhoPlan& R, int dtype) {
  if (R.generic) return gen_ws_layout(R, dtype).total;
  size_t t = ws_layout(R.G, dtype).total;
  if (R.perm) t += align256((size_t)R.G.n * 8) + align256((size_t)R.G.p * 8);
  return t;
}

size_t glam_rho_workspace_size(int d, const int64_t* n, const int64_t* p, int dtype) {
  RhoPlan R;
  if (plan_rho(d, n, p, dtype, &R, true) != GLAM_OK) return 0;
  return rho_ws_total(R, dtype);
}

// the factor list of the lifted d = 3 model (d = 2: the middle factor is a 1 in the workspace)
static int lift_factors(int d, const void* const* X, char* ws, const WsLayout& W, int dtype, hipStream_t s,
                        const void** X3) {
  if (!X || !X[0] || !X[1] || (d == 3 && !X[2])) return fail(GLAM_EINVAL, "NULL pointer");
  if (d == 3) {
    X3[0] = X[0]; X3[1] = X[1]; X3[2] = X[2];
    return GLAM_OK;
  }
  HIPCHK(launch_set_one(dtype, ws + W.unit, s));
  X3[0] = X[0]; X3[1] = ws + W.unit; X3[2] = X[1];
  return GLAM_OK;
}

// the generic chain: three GEMMs per direction in the caller's (cyclic) mode order
static int gen_factors(int d, const void* const* X, char* ws, const GenWs& W, int dtype, hipStream_t s,
                       const void** X3) {
  if (!X || !X[0] || !X[1] || (d == 3 && !X[2])) return fail(GLAM_EINVAL, "NULL pointer");
  if (d == 3) {
    X3[0] = X[0]; X3[1] = X[1]; X3[2] = X[2];
    return GLAM_OK;
  }
  HIPCHK(launch_set_one(dtype, ws + W.unit, s));
  X3[0] = X[0]; X3[1] = ws + W.unit; X3[2] = X[1];
  return GLAM_OK;
}
static int gen_forward(const RhoPlan& R, int d, const void* const* X_in, const void* Theta, void* Eta, int dtype,
                       char* ws, hipStream_t s) {
  const GenWs W = gen_ws_layout(R, dtype);
  const void* X[3];
  int st = gen_factors(d, X_in, ws, W, dtype, s, X);
  if (st) return st;
  const void* XT[3];
  for (int j = 0; j < 3; ++j) {
    HIPCHK(launch_gen_transpose_same(dtype, R.n[j], R.p[j], X[j], ws + W.xt[j], s));
    XT[j] = ws + W.xt[j];
  }
  HIPCHK(general_forward(dtype, R.n, R.p, XT, Theta, ws + W.t1, ws + W.t2, Eta, false, s));
  return GLAM_OK;
}
static int gen_adjoint(const RhoPlan& R, int d, const void* const* X_in, const void* U, void* Out, int dtype, char* ws,
                       hipStream_t s) {
  const GenWs W = gen_ws_layout(R, dtype);
  const void* X[3];
  int st = gen_factors(d, X_in, ws, W, dtype, s, X);
  if (st) return st;
  HIPCHK(general_adjoint(dtype, R.n, R.p, X, U, ws + W.t1, ws + W.t2, Out, s));
  return GLAM_OK;
}

int glam_rho_forward(int d, const int64_t* n, const int64_t* p, const void* const* X_in, const void* Theta_in, void* Eta_out,
                     int dtype, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  RhoPlan R;
  int st = plan_rho(d, n, p, dtype, &R, true);
  if (st) return st;
  if (R.generic) {
    if (!Theta_in || !Eta_out || !workspace) return fail(GLAM_EINVAL, "NULL pointer");
    if (ws_bytes < rho_ws_total(R, dtype)) return fail(GLAM_EINVAL, "workspace too small");
    return gen_forward(R, d, X_in, Theta_in, Eta_out, dtype, (char*)workspace, (hipStream_t)stream);
  }
  const Geom& G = R.G;
  if (!Theta_in || !Eta_out || !workspace) return fail(GLAM_EINVAL, "NULL pointer");
  if (ws_bytes < rho_ws_total(R, dtype)) return fail(GLAM_EINVAL, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const WsLayout W = ws_layout(G, dtype);
  char* ws = (char*)workspace;
  const void* Xl[3];
  st = lift_factors(d, X_in, ws, W, dtype, s, Xl);
  if (st) return st;
  const void* X[3] = {Xl[R.q[0]], Xl[R.q[1]], Xl[R.q[2]]};
  const size_t es = dt_size(dtype), oes = dtype == DT_F64 ? 8 : 4;
  const void* Theta = Theta_in;
  void* Eta = Eta_out;
  char* reg_n = ws + W.total;                             // eta in the order that runs
  char* reg_p = reg_n + align256((size_t)G.n * 8);        // Theta in that order
  if (R.perm) {
    HIPCHK(launch_permute3_es((int)es, Theta_in, reg_p, R.p, R.q, s));
    Theta = reg_p;
    Eta = reg_n;
  }
  HIPCHK(launch_pack(dtype, dtype, Theta, G.p3, G.P12, G.P12, 1, ws + W.inc, s));
  HIPCHK(launch_pack(dtype, dtype, X[2], G.p3, G.n3, G.n3, 1, ws + W.x3f, s));
  FwdParams F{};
  F.G = G; F.theta = ws + W.inc; F.X3f = ws + W.x3f; F.T1 = ws + W.t1; F.iter = nullptr;
  HIPCHK(launch_slab_fwd(dtype, F, s));
  SlabParams S{};
  HIPCHK(launch_pack_chain_image(dtype, dtype, G, X[0], X[1], ws + W.img, s, chain_image_need(dtype, SM_FWD_STD, G)));
  S.G = G; S.img = ws + W.img; S.T1 = ws + W.t1; S.eta_out = Eta;
  HIPCHK(launch_slab_chain(dtype, SM_FWD_STD, S, nullptr, s));
  if (R.perm) {   // back to the caller's order
    int qi[3];
    for (int k = 0; k < 3; ++k) qi[R.q[k]] = k;
    const int64_t nr[3] = {G.n1, G.n2, G.n3};
    HIPCHK(launch_permute3_es((int)oes, reg_n, Eta_out, nr, qi, s));
  }
  return GLAM_OK;
}

int glam_rho_forward_static(int d, const int64_t* n, const int64_t* p, const void* const* X, const void* Theta,
                            void* Eta, int dtype, void* stream) {
  g_err.clear();
  RhoPlan R;
  const int st = plan_rho(d, n, p, dtype, &R, true);
  if (st) return st;
  const size_t need = rho_ws_total(R, dtype);
  if (need > (size_t)GLAM_STATIC_SCRATCH_BYTES)
    return fail(GLAM_EINVAL, "these sizes need " + std::to_string(need) + " bytes of workspace, more than the " +
                                 std::to_string((size_t)GLAM_STATIC_SCRATCH_BYTES) + "-byte static scratch");
  void* ws = nullptr;
  const int sa = scratch_address(&ws);
  if (sa) return sa;
  // the same kernels as glam_rho_forward: every workspace region it reads is written first on
  // the stream (packing zero-fills the padding), so the previous call's contents do not matter
  return glam_rho_forward(d, n, p, X, Theta, Eta, dtype, ws, (size_t)GLAM_STATIC_SCRATCH_BYTES, stream);
}

int glam_rho_adjoint(int d, const int64_t* n, const int64_t* p, const void* const* X_in, const void* U_in, void* Out_p,
                     int dtype, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  RhoPlan R;
  int st = plan_rho(d, n, p, dtype, &R, true);
  if (st) return st;
  if (R.generic) {
    if (!U_in || !Out_p || !workspace) return fail(GLAM_EINVAL, "NULL pointer");
    if (ws_bytes < rho_ws_total(R, dtype)) return fail(GLAM_EINVAL, "workspace too small");
    return gen_adjoint(R, d, X_in, U_in, Out_p, dtype, (char*)workspace, (hipStream_t)stream);
  }
  const Geom& G = R.G;
  if (!U_in || !Out_p || !workspace) return fail(GLAM_EINVAL, "NULL pointer");
  if (ws_bytes < rho_ws_total(R, dtype)) return fail(GLAM_EINVAL, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const WsLayout W = ws_layout(G, dtype);
  char* ws = (char*)workspace;
  const void* Xl[3];
  st = lift_factors(d, X_in, ws, W, dtype, s, Xl);
  if (st) return st;
  const void* X[3] = {Xl[R.q[0]], Xl[R.q[1]], Xl[R.q[2]]};
  const size_t es = dt_size(dtype), oes = dtype == DT_F64 ? 8 : 4;
  const void* U = U_in;
  void* Out = Out_p;
  char* reg_n = ws + W.total;                             // U in the order that runs
  char* reg_p = reg_n + align256((size_t)G.n * 8);        // the output in that order
  if (R.perm) {
    HIPCHK(launch_permute3_es((int)es, U_in, reg_n, R.n, R.q, s));
    U = reg_n;
    Out = reg_p;
  }
  HIPCHK(launch_pack(dtype, dtype, X[2], G.n3, G.p3, 1, G.n3, ws + W.x3a, s));
  HIPCHK(launch_zero(ws + W.s2 + (size_t)(G.KBN3 - 1) * 16 * G.P12 * es, (size_t)16 * G.P12 * es, s));
  SlabParams S{};
  HIPCHK(launch_pack_chain_image(dtype, dtype, G, X[0], X[1], ws + W.img, s, chain_image_need(dtype, SM_ADJ_STD, G)));
  S.G = G; S.img = ws + W.img; S.S2 = ws + W.s2; S.u_in = U;
  HIPCHK(launch_slab_chain(dtype, SM_ADJ_STD, S, nullptr, s));
  AdjParams A{};
  A.G = G; A.S2 = ws + W.s2; A.X3a = ws + W.x3a; A.out = Out; A.scale = 1.0;
  HIPCHK(launch_slab_adj(dtype, EPI_STORE, A, nullptr, s));
  if (R.perm) {   // back to the caller's order
    int qi[3];
    for (int k = 0; k < 3; ++k) qi[R.q[k]] = k;
    const int64_t pr[3] = {G.p1, G.p2, G.p3};
    HIPCHK(launch_permute3_es((int)oes, reg_p, Out_p, pr, qi, s));
  }
  return GLAM_OK;
}

// NLL workspace: the rho layout of the order that runs, then (reordered problems) regions for
// Y (n FP64), beta and the gradient (p elements of 8 bytes each) in that order.
struct NllRegions {
  char *y, *beta, *grad;
};
static size_t nll_extra_bytes(const RhoPlan& R) {
  return R.perm ? align256((size_t)R.G.n * 8) + 2 * align256((size_t)R.G.p * 8) : 0;
}
static NllRegions nll_regions(const RhoPlan& R, char* base) {
  NllRegions g;
  g.y = base;
  g.beta = g.y + align256((size_t)R.G.n * 8);
  g.grad = g.beta + align256((size_t)R.G.p * 8);
  return g;
}
static void nll_factors(const RhoPlan& R, const void* const* X, const void** Xr) {
  for (int k = 0; k < 3; ++k) Xr[k] = X[R.q[k]];
}
// gradient of the order that ran -> the caller's order
static hipError_t nll_grad_back(const RhoPlan& R, int dtype, const void* gr, void* grad, hipStream_t s) {
  int qi[3];
  for (int k = 0; k < 3; ++k) qi[R.q[k]] = k;
  const int64_t pr[3] = {R.G.p1, R.G.p2, R.G.p3};
  return launch_permute3_es(dtype == DT_F64 ? 8 : 4, gr, grad, pr, qi, s);
}

size_t glam_nll_workspace_size(const int64_t* n, const int64_t* p, int dtype) {
  RhoPlan R;
  if (plan_rho(3, n, p, dtype, &R) != GLAM_OK) return 0;
  return ws_layout(R.G, dtype).total + nll_extra_bytes(R);
}

// Shared forward part of the NLL entry points: eta = H(beta) inside slab_chain.
static int nll_prepare(const Geom& G, const void* const* X, const void* beta, int dtype, char* ws, const WsLayout& W,
                       hipStream_t s) {
  const size_t es = dt_size(dtype);
  HIPCHK(launch_pack(dtype, dtype, beta, G.p3, G.P12, G.P12, 1, ws + W.inc, s));
  HIPCHK(launch_pack(dtype, dtype, X[2], G.p3, G.n3, G.n3, 1, ws + W.x3f, s));
  HIPCHK(launch_pack_chain_image(dtype, dtype, G, X[0], X[1], ws + W.img, s,
                                 chain_image_need(dtype, SM_NLL_FWD, G) | chain_image_need(dtype, SM_NLL_BWD, G)));
  FwdParams F{};
  F.G = G; F.theta = ws + W.inc; F.X3f = ws + W.x3f; F.T1 = ws + W.t1;
  HIPCHK(launch_slab_fwd(dtype, F, s));
  return GLAM_OK;
}

int glam_poisson_nll_forward(const int64_t* n, const int64_t* p, const void* const* X_in, const void* beta_in,
                             const double* Y_in, double* loss, int dtype, void* workspace, size_t ws_bytes,
                             void* stream) {
  g_err.clear();
  RhoPlan R;
  int st = plan_rho(3, n, p, dtype, &R);
  if (st) return st;
  const Geom& G = R.G;
  if (!X_in || !X_in[0] || !X_in[1] || !X_in[2] || !beta_in || !Y_in || !loss || !workspace)
    return fail(GLAM_EINVAL, "NULL pointer");
  if (ws_bytes < glam_nll_workspace_size(n, p, dtype)) return fail(GLAM_EINVAL, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const WsLayout W = ws_layout(G, dtype);
  const void* X[3];
  nll_factors(R, X_in, X);
  const void* beta = beta_in;
  const double* Y = Y_in;
  if (R.perm) {   // Y and beta in the order that runs (the loss is the same)
    const NllRegions g = nll_regions(R, ws + W.total);
    HIPCHK(launch_permute3_es((int)dt_size(dtype), beta_in, g.beta, R.p, R.q, s));
    HIPCHK(launch_permute3_es(8, Y_in, g.y, R.n, R.q, s));
    beta = g.beta;
    Y = (const double*)g.y;
  }
  st = nll_prepare(G, X, beta, dtype, ws, W, s);
  if (st) return st;
  double* part = (double*)(ws + W.part);
  SlabParams S{};
  S.G = G; S.img = ws + W.img; S.T1 = ws + W.t1; S.y_std = Y; S.partials = part;
  int nb = 0;
  HIPCHK(launch_slab_chain(dtype, SM_NLL_FWD, S, &nb, s));
  const int ops[1] = {0};
  HIPCHK(launch_reduce_strided(part, nb, 2, 1, ops, 1.0 / (double)G.n, loss, s));
  return GLAM_OK;
}

int glam_poisson_nll_backward(const int64_t* n, const int64_t* p, const void* const* X_in, const void* beta_in,
                              const double* Y_in, const double* gscale, void* grad_out, int dtype, void* workspace,
                              size_t ws_bytes, void* stream) {
  g_err.clear();
  RhoPlan R;
  int st = plan_rho(3, n, p, dtype, &R);
  if (st) return st;
  const Geom& G = R.G;
  if (!X_in || !X_in[0] || !X_in[1] || !X_in[2] || !beta_in || !Y_in || !grad_out || !workspace)
    return fail(GLAM_EINVAL, "NULL pointer");
  if (ws_bytes < glam_nll_workspace_size(n, p, dtype)) return fail(GLAM_EINVAL, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const WsLayout W = ws_layout(G, dtype);
  const size_t es = dt_size(dtype);
  const void* X[3];
  nll_factors(R, X_in, X);
  const void* beta = beta_in;
  const double* Y = Y_in;
  void* grad = grad_out;
  const NllRegions g = nll_regions(R, ws + W.total);
  if (R.perm) {
    HIPCHK(launch_permute3_es((int)es, beta_in, g.beta, R.p, R.q, s));
    HIPCHK(launch_permute3_es(8, Y_in, g.y, R.n, R.q, s));
    beta = g.beta;
    Y = (const double*)g.y;
    grad = g.grad;
  }
  st = nll_prepare(G, X, beta, dtype, ws, W, s);
  if (st) return st;
  HIPCHK(launch_pack(dtype, dtype, X[2], G.n3, G.p3, 1, G.n3, ws + W.x3a, s));
  HIPCHK(launch_zero(ws + W.s2 + (size_t)(G.KBN3 - 1) * 16 * G.P12 * es, (size_t)16 * G.P12 * es, s));
  SlabParams S{};
  S.G = G; S.img = ws + W.img; S.T1 = ws + W.t1; S.S2 = ws + W.s2; S.y_std = Y;
  S.partials = (double*)(ws + W.part);
  HIPCHK(launch_slab_chain(dtype, SM_NLL_BWD, S, nullptr, s));
  AdjParams A{};
  A.G = G; A.S2 = ws + W.s2; A.X3a = ws + W.x3a; A.out = grad; A.scale = 1.0 / (double)G.n; A.gscale_dev = gscale;
  A.s2_kb4 = chain_s2_kb4(dtype, SM_NLL_BWD, G);
  HIPCHK(launch_slab_adj(dtype, EPI_STORE, A, nullptr, s));
  if (R.perm) HIPCHK(nll_grad_back(R, dtype, g.grad, grad_out, s));
  return GLAM_OK;
}

// ---------------------------------------------------------------------------
// NLL with the factors and counts packed once (the workspace keeps them between calls)
// ---------------------------------------------------------------------------
// Layout: the rho workspace, then the counts: tiled FP32 for the one-wave-per-slab kernel,
// else an FP64 copy in the standard layout.
// A reordered problem (see plan_rho) also has the n/p regions of the one-shot calls after it.
struct NllPacked {
  RhoPlan R;
  WsLayout W;
  size_t y, extra, total;
  bool tiled;
};
static NllPacked nll_packed_layout(const RhoPlan& R, int dt) {
  NllPacked L;
  L.R = R;
  L.W = ws_layout(R.G, dt);
  L.tiled = chain_image_need(dt, SM_NLL_FWD, R.G) == PACK_WAVE;
  L.y = L.W.total;
  L.extra = L.y + align256(L.tiled ? (size_t)R.G.nint * sizeof(float) : (size_t)R.G.n * sizeof(double));
  L.total = L.extra + nll_extra_bytes(R);
  return L;
}

size_t glam_nll_packed_workspace_size(const int64_t* n, const int64_t* p, int dtype) {
  RhoPlan R;
  if (plan_rho(3, n, p, dtype, &R) != GLAM_OK) return 0;
  return nll_packed_layout(R, dtype).total;
}

int glam_poisson_nll_pack(const int64_t* n, const int64_t* p, const void* const* X_in, const double* Y_in, int dtype,
                          void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  RhoPlan R;
  int st = plan_rho(3, n, p, dtype, &R);
  if (st) return st;
  const Geom& G = R.G;
  if (!X_in || !X_in[0] || !X_in[1] || !X_in[2] || !Y_in || !workspace) return fail(GLAM_EINVAL, "NULL pointer");
  if (ws_bytes < glam_nll_packed_workspace_size(n, p, dtype)) return fail(GLAM_EINVAL, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const NllPacked L = nll_packed_layout(R, dtype);
  const WsLayout& W = L.W;
  const void* X[3];
  nll_factors(R, X_in, X);
  const double* Y = Y_in;
  if (R.perm) {   // the counts in the order that runs, then packed from there
    const NllRegions g = nll_regions(R, ws + L.extra);
    HIPCHK(launch_permute3_es(8, Y_in, g.y, R.n, R.q, s));
    Y = (const double*)g.y;
  }
  const size_t es = dt_size(dtype);
  HIPCHK(launch_pack(dtype, dtype, X[2], G.p3, G.n3, G.n3, 1, ws + W.x3f, s));
  HIPCHK(launch_pack(dtype, dtype, X[2], G.n3, G.p3, 1, G.n3, ws + W.x3a, s));
  HIPCHK(launch_pack_chain_image(dtype, dtype, G, X[0], X[1], ws + W.img, s,
                                 chain_image_need(dtype, SM_NLL_FWD, G) | chain_image_need(dtype, SM_NLL_BWD, G)));
  HIPCHK(launch_zero(ws + W.s2 + (size_t)(G.KBN3 - 1) * 16 * G.P12 * es, (size_t)16 * G.P12 * es, s));
  if (L.tiled) HIPCHK(launch_to_tiled_f32(G, Y, (float*)(ws + L.y), s));
  else HIPCHK(hipMemcpyAsync(ws + L.y, Y, (size_t)G.n * sizeof(double), hipMemcpyDeviceToDevice, s));
  return GLAM_OK;
}

// checks shared by the packed entry points; eta = H(beta) into T1 of the workspace
static int nll_packed_begin(const int64_t* n, const int64_t* p, const void* beta_in, int dtype, void* workspace,
                            size_t ws_bytes, hipStream_t s, Geom* G, NllPacked* L) {
  RhoPlan R;
  int st = plan_rho(3, n, p, dtype, &R);
  if (st) return st;
  *G = R.G;
  if (!beta_in || !workspace) return fail(GLAM_EINVAL, "NULL pointer");
  if (ws_bytes < glam_nll_packed_workspace_size(n, p, dtype)) return fail(GLAM_EINVAL, "workspace too small");
  *L = nll_packed_layout(R, dtype);
  char* ws = (char*)workspace;
  const void* beta = beta_in;
  if (R.perm) {
    const NllRegions g = nll_regions(R, ws + L->extra);
    HIPCHK(launch_permute3_es((int)dt_size(dtype), beta_in, g.beta, R.p, R.q, s));
    beta = g.beta;
  }
  HIPCHK(launch_pack(dtype, dtype, beta, G->p3, G->P12, G->P12, 1, ws + L->W.inc, s));
  FwdParams F{};
  F.G = *G; F.theta = ws + L->W.inc; F.X3f = ws + L->W.x3f; F.T1 = ws + L->W.t1;
  HIPCHK(launch_slab_fwd(dtype, F, s));
  return GLAM_OK;
}

int glam_poisson_nll_forward_packed(const int64_t* n, const int64_t* p, const void* beta, double* loss, int dtype,
                                    void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!loss) return fail(GLAM_EINVAL, "NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  Geom G;
  NllPacked L;
  int st = nll_packed_begin(n, p, beta, dtype, workspace, ws_bytes, s, &G, &L);
  if (st) return st;
  char* ws = (char*)workspace;
  double* part = (double*)(ws + L.W.part);
  SlabParams S{};
  S.G = G; S.img = ws + L.W.img; S.T1 = ws + L.W.t1; S.partials = part;
  if (L.tiled) S.y_tiled = (const float*)(ws + L.y);
  else S.y_std = (const double*)(ws + L.y);
  int nb = 0;
  HIPCHK(launch_slab_chain(dtype, SM_NLL_FWD, S, &nb, s));
  const int ops[1] = {0};
  HIPCHK(launch_reduce_strided(part, nb, 2, 1, ops, 1.0 / (double)G.n, loss, s));
  return GLAM_OK;
}

int glam_poisson_nll_backward_packed(const int64_t* n, const int64_t* p, const void* beta, const double* gscale,
                                     void* grad_out, int dtype, void* workspace, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!grad_out) return fail(GLAM_EINVAL, "NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  Geom G;
  NllPacked L;
  int st = nll_packed_begin(n, p, beta, dtype, workspace, ws_bytes, s, &G, &L);
  if (st) return st;
  char* ws = (char*)workspace;
  SlabParams S{};
  S.G = G; S.img = ws + L.W.img; S.T1 = ws + L.W.t1; S.S2 = ws + L.W.s2;
  S.partials = (double*)(ws + L.W.part);
  if (L.tiled) S.y_tiled = (const float*)(ws + L.y);
  else S.y_std = (const double*)(ws + L.y);
  HIPCHK(launch_slab_chain(dtype, SM_NLL_BWD, S, nullptr, s));
  AdjParams A{};
  const NllRegions g = nll_regions(L.R, ws + L.extra);
  void* grad = L.R.perm ? (void*)g.grad : grad_out;
  A.G = G; A.S2 = ws + L.W.s2; A.X3a = ws + L.W.x3a; A.out = grad; A.scale = 1.0 / (double)G.n; A.gscale_dev = gscale;
  A.s2_kb4 = chain_s2_kb4(dtype, SM_NLL_BWD, G);
  HIPCHK(launch_slab_adj(dtype, EPI_STORE, A, nullptr, s));
  if (L.R.perm) HIPCHK(nll_grad_back(L.R, dtype, g.grad, grad_out, s));
  return GLAM_OK;
}

}  // extern "C"
