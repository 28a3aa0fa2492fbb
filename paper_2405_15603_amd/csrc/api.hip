// Host side of the C ABI (include/kfac_pinn.h): context, workspace plan, and the
// order of the launches that make up one KFAC step (Algorithm 1).  Everything
// is enqueued on the context's stream; nothing here reads device data back
// except kfac_pinn_sync.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "common.h"
#include "fwdlap.h"
#include "kfac_pinn.h"
#include "launch.h"

using namespace kp;

static thread_local std::string g_last_error;
void kp_set_last_error(const char* msg, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "%s (%s:%d)", msg, file, line);
  g_last_error = buf;
}
#define KP_ARG(cond, msg)                                  \
  do {                                                     \
    if (!(cond)) {                                         \
      kp_set_last_error(msg, __FILE__, __LINE__);          \
      return KP_ERR_ARG;                                   \
    }                                                      \
  } while (0)
#define KP_TRY(expr)                                       \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) {                                \
      kp_set_last_error(hipGetErrorString(_e), __FILE__, __LINE__); \
      return KP_ERR_HIP;                                   \
    }                                                      \
  } while (0)

namespace {

constexpr int kMaxLayers = 8;
constexpr int kMaxCand = 64;
constexpr int kMaxSplits = 64;
constexpr int kJacobiSweeps = 20;
constexpr long kMaxGramianParams = 16384;
// Jacobi starts from the previous call's eigenvectors except on every
// kEigRefresh-th call (and the first), which starts from the identity so that
// rounding in the carried rotations cannot accumulate without bound.
constexpr int kEigRefresh = 1000;

struct Slabs {            // one term (interior or boundary); rows are s-major (s*N + p)
  int S = 1, nd = 0, has_lap = 0, cap = 0;   // rows per point, derivative rows, capacity (points)
  bool store = true;
  std::vector<void*> zin;                    // stored: layer inputs Z~^(l) (l = 0..L-1)
  std::vector<void*> pre;                    // stored: hidden pre-activations (l = 0..L-2)
  std::vector<void*> g;                      // stored: output gradients (l = 0..L-1)
  void* zr[2] = {nullptr, nullptr};          // recompute: layer inputs (ping-pong)
  void* prer = nullptr;                      // recompute: one hidden pre-activation slab
  void* gr[2] = {nullptr, nullptr};          // recompute: output gradients (ping-pong)
  std::vector<void*> sq;                     // per hidden layer: N x h sum of squares
  void* u = nullptr;                         // network output rows (compute type, R)
  double* r = nullptr;                       // residual per point
  float* rf = nullptr;                       // its FP32 copy
  void* zin_at(int l) const { return store ? zin[l] : zr[l & 1]; }
  void* g_at(int l) const { return store ? g[l] : gr[l & 1]; }
  void* pre_at(int l) const { return store ? pre[l] : prer; }
};

}  // namespace

struct kfac_pinn_ctx {
  int L = 0, d = 0;
  std::vector<int> w;
  int time_coord = -1;
  double c_t = 0.0, c_lap = -1.0;
  // first-order terms of the interior residual (Section 3.3; zero for linear PDEs):
  // sum_{i in mask} (c_x x_i d_i u + c_g (d_i u)^2) + c_0
  double c_x = 0.0, c_g = 0.0, c_0 = 0.0;
  bool nonlinear = false;
  int precision = KP_F32;
  Prec pp = P_F32;          // parameters and points
  Prec sp = P_F32;          // curvature slabs
  Prec lp = P_F32;          // line-search slabs
  Prec wp = P_F32;          // product-layout weights
  int cmode = M_F32;        // curvature products
  int lmode = M_F32;        // line-search products
  size_t esz_p = 4, esz_s = 4, esz_l = 4, esz_c = 4, esz_w = 4;
  int max_i = 0, max_b = 0;
  size_t ws_limit = 0;
  hipStream_t st = nullptr;
  long D = 0;
  void* qbuf = nullptr;     // input layer: sums of squared weights and transposed weights
  NetDesc nd{};
  std::vector<long> off, ldz, ldp, ldg;
  long ldz_max = 0, ldp_max = 0;

  // device buffers: the pointer handed out, the allocation it lives in and its size;
  // with guards (KFAC_PINN_GUARD_KB) the allocation has `guard` pattern bytes on
  // either side of the buffer
  struct Alloc { void* user; void* base; size_t bytes; };
  std::vector<Alloc> allocs;
  size_t guard = 0;
  int max_sweeps = kJacobiSweeps;
  float* wts = nullptr;     // weights of the derivative rows' squares (mask or eigenvalues of C)
  double* wts64 = nullptr;  // the same in FP64
  double* dirs = nullptr;   // input directions (rows: eigenvectors of C), nullptr = unit vectors
  void *w_hi = nullptr, *w_lo = nullptr;
  void* theta_trial = nullptr;
  Slabs si, sb;
  void* tab = nullptr;                 // finishing-pass tables (compute type)
  long tab_stride = 0;                 // elements per table plane (max N * h)
  void* ls_z[2] = {nullptr, nullptr};
  void* ls_u = nullptr;
  // boundary line-search slabs, one per layer input: their bias and padding
  // columns are written once at creation (one row per point, so they do not depend
  // on the point count), and the paired launches store only the product columns
  void* ls_zb[kMaxLayers] = {};
  void* ls_ub = nullptr;
  double* partial = nullptr;
  int partial_n = 0;
  double* loss = nullptr;              // [0] L_int [1] L_bnd [2..] candidates
  int last_ncand = 0;
  std::vector<double*> F[2][2];        // F[term][side][layer]
  void* part = nullptr;
  float* wsc = nullptr;                 // FP16 row-weight scale (2 floats)
  double* grad = nullptr;
  double* Delta = nullptr;
  void* dhat = nullptr;
  void* delta = nullptr;
  std::vector<EigProblem> probs;        // layer l: 2l side A, 2l + 1 side B
  EigProblem* probs_dev = nullptr;
  EigGroups eg;                         // Jacobi groups; side streams made on first use
  bool eg_streams = false;
  // Line-search lanes: odd candidates run on the first side stream with their own
  // buffers (lane 1), made on the first step that uses them outside a capture.
  int ls_lanes = 2;
  struct LsLane {
    bool ready = false;
    hipStream_t st = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    void* theta_trial = nullptr;
    void* w_hi = nullptr;
    void* ls_z[2] = {nullptr, nullptr};
    void* ls_u = nullptr;
    void* ls_zb[kMaxLayers] = {};
    void* ls_ub = nullptr;
    void* tab = nullptr;
    double* partial = nullptr;
    void* qbuf = nullptr;
  } ls1;
  size_t w_bytes = 0;                   // product-layout weight copy
  G64* kdesc = nullptr;
  int k_mmax = 0, k_nmax = 0;
  int* ctl = nullptr;                  // [0] status [1] step [4..7] alpha, mu [8..] Jacobi flags
  // KFAC*: per-point Jacobian-vector products (term, direction, point) and the
  // per-tile partial sums they are gathered from
  double* jv = nullptr;
  long jv_ld = 0;
  void* jvp_part = nullptr;
  int last_n[2] = {0, 0};   // point counts of the last curvature pass (interior, boundary)
  // the batch's grouped factor products: the curvature pass leaves the products
  // to a grouped launch over every instance
  bool defer_products = false;
  // measurement: launches of one kernel class bracketed by events
  int tm_cls = -1;
  std::vector<hipEvent_t> tm_ev;
  int tm_used = 0;
  double tm_flops = 0.0, tm_bytes = 0.0;
  long tm_launches = 0;
};

namespace {

constexpr unsigned char kGuardByte = 0xA5;

hipError_t dmalloc(kfac_pinn_ctx* c, void** p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  const size_t g = c->guard;
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, bytes + 2 * g);
  if (e != hipSuccess) return e;
  *p = (char*)base + g;
  c->allocs.push_back({*p, base, bytes});
  if (g > 0 && ((e = hipMemset(base, kGuardByte, g)) != hipSuccess ||
                (e = hipMemset((char*)*p + bytes, kGuardByte, g)) != hipSuccess))
    return e;
  return hipMemset(*p, 0, bytes);
}

// A = V diag(w) V^T for a small symmetric matrix (row-major n x n, host), by
// cyclic Jacobi rotations (tan of the rotation from the textbook quadratic
// t^2 + 2 theta t - 1 = 0) until the off-diagonal part is below 1e-32 of the
// squared Frobenius norm.  A row and column that are zero are never rotated, so
// e_k stays an eigenvector exactly.  The matrix is symmetrised first.
void eig_sym_host(int n, const double* A0, std::vector<double>& V, std::vector<double>& w) {
  std::vector<double> A((size_t)n * n);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) A[(size_t)i * n + j] = 0.5 * (A0[(size_t)i * n + j] + A0[(size_t)j * n + i]);
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; i++) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0, fro = 0.0;
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) {
        fro += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (off <= 1e-32 * fro) break;
    for (int p = 0; p < n - 1; p++)
      for (int q = p + 1; q < n; q++) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        const double th = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; k++) {   // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = cs * akp - sn * akq;
          a(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; k++) {   // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = cs * apk - sn * aqk;
          a(q, k) = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; k++) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = cs * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; i++) w[i] = a(i, i);
}

void dfree(kfac_pinn_ctx* c, void* user) {
  for (size_t i = 0; i < c->allocs.size(); i++)
    if (c->allocs[i].user == user) {
      (void)hipFree(c->allocs[i].base);
      c->allocs.erase(c->allocs.begin() + (long)i);
      return;
    }
}

size_t slab_bytes(const kfac_pinn_ctx* c, const Slabs& s, bool store) {
  const size_t R = (size_t)s.cap * s.S;
  size_t b = R * c->esz_c;   // output rows
  if (store) {
    for (int l = 0; l < c->L; l++) {
      b += R * (c->ldz[l] + c->ldg[l]) * c->esz_s;
      if (l + 1 < c->L) b += R * c->ldp[l] * c->esz_c;
    }
  } else {
    b += R * (2 * c->ldz_max * c->esz_s + c->ldp_max * c->esz_c + 2 * c->ldp_max * c->esz_s);
  }
  return b;
}

hipError_t alloc_slabs(kfac_pinn_ctx* c, Slabs& s) {
  const size_t R = (size_t)s.cap * s.S;
  hipError_t e;
  if (s.store) {
    s.zin.assign(c->L, nullptr);
    s.pre.assign(c->L, nullptr);
    s.g.assign(c->L, nullptr);
    for (int l = 0; l < c->L; l++) {
      if ((e = dmalloc(c, &s.zin[l], R * c->ldz[l] * c->esz_s)) != hipSuccess) return e;
      if ((e = dmalloc(c, &s.g[l], R * c->ldg[l] * c->esz_s)) != hipSuccess) return e;
      if (l + 1 < c->L &&
          (e = dmalloc(c, &s.pre[l], R * c->ldp[l] * c->esz_c)) != hipSuccess)
        return e;
    }
  } else {
    for (int k = 0; k < 2; k++) {
      if ((e = dmalloc(c, &s.zr[k], R * c->ldz_max * c->esz_s)) != hipSuccess) return e;
      if ((e = dmalloc(c, &s.gr[k], R * c->ldp_max * c->esz_s)) != hipSuccess) return e;
    }
    if ((e = dmalloc(c, &s.prer, R * c->ldp_max * c->esz_c)) != hipSuccess) return e;
  }
  s.sq.assign(c->L, nullptr);
  if (s.has_lap)
    for (int l = 0; l + 1 < c->L; l++)
      if ((e = dmalloc(c, &s.sq[l], (size_t)s.cap * c->w[l + 1] * c->esz_c)) != hipSuccess)
        return e;
  if ((e = dmalloc(c, &s.u, R * c->esz_c)) != hipSuccess) return e;
  // residuals in FP64, then their FP32 copy (the BF16x3 gradient product reads it)
  if ((e = dmalloc(c, (void**)&s.r, sizeof(double) * (s.cap > 0 ? s.cap : 1))) != hipSuccess)
    return e;
  return dmalloc(c, (void**)&s.rf, sizeof(float) * (s.cap > 0 ? s.cap : 1));
}

inline char* wptr(const void* base, long elems, size_t esz) { return (char*)base + elems * esz; }

// kernel classes for timing
enum { KC_LAYER_GEMM = 0, KC_FACTOR_GEMM = 1, KC_INVERT = 2, KC_ACT = 3, KC_LS_LAYER = 4 };

int tm_begin(kfac_pinn_ctx* c, int cls) {
  if (c->tm_cls != cls) return -1;
  if (c->tm_used + 2 > (int)c->tm_ev.size()) {
    for (int k = 0; k < 256; k++) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      c->tm_ev.push_back(e);
    }
  }
  const int idx = c->tm_used;
  c->tm_used += 2;
  (void)hipEventRecord(c->tm_ev[idx], c->st);
  return idx;
}
void tm_end(kfac_pinn_ctx* c, int idx, double flops, double bytes) {
  if (idx < 0) return;
  (void)hipEventRecord(c->tm_ev[idx + 1], c->st);
  c->tm_flops += flops;
  c->tm_bytes += bytes;
  c->tm_launches += 1;
}

int lap_row_of(const Slabs& s) { return s.has_lap ? s.S - 1 : -1; }
int time_row_of(const kfac_pinn_ctx* c, const Slabs& s) {
  return (s.has_lap && c->time_coord >= 0 && c->c_t != 0.0) ? 1 + c->time_coord : -1;
}

// Where one forward pass reads its weights and writes its slabs.
struct FwdTarget {
  int mode;
  Prec zp;                      // slab storage
  size_t zesz;
  const void* theta;            // parameters (last layer read directly)
  std::function<void*(int)> z;  // layer-input slab of layer l
  std::function<void*(int)> pre;   // hidden pre-activations of layer l (or nullptr)
  std::function<void*(int)> sq;    // sum of squares table of layer l (or nullptr)
  void* u;                      // output rows
  int kc_layer = KC_LAYER_GEMM;  // timing class of the layer products
  bool full_input = true;        // write every row of the input slab (false: value rows)
  bool residual_rows = false;    // interior: only the output rows the residual reads
  bool narrow_pad = false;       // rows read and padded only to h + 1 rounded up to 8
};

// One hidden layer's product: its arguments, chunk count and accounting.
struct LayerLaunch {
  FwdLayerArgs a{};
  int nch = 1;
  bool input_rows = false;   // the input layer's rows without products follow
  double flops = 0.0, bytes = 0.0;
};

LayerLaunch layer_launch(kfac_pinn_ctx* c, const Slabs& s, int n, int l, int upto,
                         const FwdTarget& T) {
  const LayerDesc& ld = c->nd.l[l];
  const long R = (long)n * s.S;
  LayerLaunch L;
  FwdLayerArgs& a = L.a;
  a.zin = T.z(l);
  a.ldz = c->ldz[l];
  a.w = wptr(c->w_hi, ld.wrm, c->esz_w);
  a.w2 = (T.mode == M_BF16X3 || T.mode == M_F16) ? wptr(c->w_lo, ld.wrm, c->esz_w) : nullptr;
  a.ldw = ld.ldk_in;
  a.K = (int)ld.ldk_in;
  a.N = n;
  a.S = s.S;
  a.nd = s.nd;
  a.has_lap = s.has_lap;
  a.h_out = ld.h_out;
  a.wts = c->wts;
  a.wts64 = c->wts64;
  a.dirs = c->dirs;
  a.d = c->d;
  a.z = T.z(l + 1);
  a.ldzo = c->ldz[l + 1];
  a.pre = T.pre(l);
  a.ldp = c->ldp[l];
  const long ts = c->tab_stride;
  a.tab_t = s.has_lap ? c->tab : nullptr;
  a.tab_lap = s.has_lap ? wptr(c->tab, ts, c->esz_c) : nullptr;
  a.tab_sq = s.has_lap ? wptr(c->tab, 2 * ts, c->esz_c) : nullptr;
  a.sq_out = T.sq(l);
  if (T.narrow_pad) {
    a.kz = (int)kp_roundup(ld.h_in + 1, 8);
    a.padz = (int)kp_roundup(ld.h_out + 1, 8);
  }
  if (T.residual_rows && s.has_lap && l == c->L - 2 && upto >= c->L) {
    // the output layer reads only the time and Laplacian rows of this layer's z
    a.sparse_store = 1;
    a.keep_value = 0;
    const int tr = time_row_of(c, s);
    a.keep_lo = tr >= 0 ? tr : 1;
    a.keep_hi = tr >= 0 ? tr : 0;
  }
  // input layer: only the value row needs products (its other input rows are
  // unit vectors and zeros)
  L.input_rows = l == 0 && s.has_lap;
  a.value_only = L.input_rows ? 1 : 0;
  L.nch = L.input_rows ? 1 : fwdlap_chunks(T.mode, n, ld.h_out, s.nd, s.has_lap);
  const double Rp = L.input_rows ? (double)n : (double)R;   // rows with products
  // bytes: the input rows with products, the z rows this launch stores (the
  // Laplacian row is the finishing pass's), the weights and the finishing tables
  const double zrows =
      a.value_only ? (double)n
      : a.sparse_store ? (double)n * (a.keep_value + std::max(0, a.keep_hi - a.keep_lo + 1))
      : (s.has_lap ? (double)n * (s.S - 1) : (double)R);
  const double tabs =
      s.has_lap ? (double)n * ld.h_out * c->esz_c * (a.value_only ? 1 : 2 + L.nch) : 0.0;
  L.flops = 2.0 * Rp * ld.h_out * (ld.h_in + 1);
  L.bytes = Rp * (ld.h_in + 1) * T.zesz + zrows * ld.h_out * T.zesz +
            (double)ld.h_out * (ld.h_in + 1) * c->esz_w + tabs;
  return L;
}

// the pass after a layer product: the input layer's remaining rows, or the
// Laplacian row, bias feature and padding
hipError_t layer_finish(kfac_pinn_ctx* c, const LayerLaunch& L, const FwdTarget& T) {
  int ti = tm_begin(c, KC_ACT);
  hipError_t e = L.input_rows ? input_layer_rows(T.mode, L.a, c->qbuf, c->st)
                              : fwdlap_finish(T.mode, L.a, L.nch, c->st);
  tm_end(c, ti, 0.0, 0.0);
  return e;
}

hipError_t output_layer(kfac_pinn_ctx* c, const Slabs& s, int n, const FwdTarget& T) {
  const LayerDesc& ld = c->nd.l[c->L - 1];
  const long lz = c->ldz[c->L - 1];
  const void* wl = wptr(T.theta, ld.off, c->esz_p);
  hipError_t e;
  if (T.residual_rows && s.has_lap && c->L >= 2) {
    // only the rows the interior residual reads: the time row and the Laplacian row
    const int rows[2] = {time_row_of(c, s), lap_row_of(s)};
    for (int k = 0; k < 2; k++) {
      if (rows[k] < 0) continue;
      const long off = (long)rows[k] * n;
      if ((e = last_fwd(T.mode, wptr(T.z(c->L - 1), off * lz, T.zesz), lz, wl, ld.h_in + 1, n,
                        wptr(T.u, off, c->esz_c), c->st)) != hipSuccess)
        return e;
    }
    return hipSuccess;
  }
  return last_fwd(T.mode, T.z(c->L - 1), lz, wl, ld.h_in + 1, (long)n * s.S, T.u, c->st);
}

int input_rows_of(kfac_pinn_ctx* c, const Slabs& s, const FwdTarget& T) {
  // Only the layer products read the input slab's derivative and Laplacian rows
  // (unit vectors and zeros); the input layer handles those rows without them,
  // so a pass that needs no input-layer factors writes the value rows only.
  return (T.full_input || !s.has_lap || c->L < 2) ? s.S : 1;
}

// Forward through hidden layers [0, upto) and, when upto == L, the output layer.
hipError_t forward_run(kfac_pinn_ctx* c, const Slabs& s, const void* x, int n, int upto,
                       const FwdTarget& T) {
  hipError_t e;
  if ((e = input_slab(T.zp, x, n, c->d, input_rows_of(c, s, T), c->dirs, T.z(0), c->ldz[0],
                      c->st)) !=
      hipSuccess)
    return e;
  const int nh = upto < c->L ? upto : c->L - 1;
  for (int l = 0; l < nh; l++) {
    const LayerLaunch L = layer_launch(c, s, n, l, upto, T);
    int ti = tm_begin(c, T.kc_layer);
    if ((e = fwdlap_main(T.mode, L.a, L.nch, c->st)) != hipSuccess) return e;
    tm_end(c, ti, L.flops, L.bytes);
    if ((e = layer_finish(c, L, T)) != hipSuccess) return e;
  }
  if (upto >= c->L) return output_layer(c, s, n, T);
  return hipSuccess;
}

// The interior and boundary forwards of one line-search candidate through the
// hidden layers, each layer's two products in one launch (the boundary tiles
// fill the interior launch's last round); the output layer is the loss kernel's.
hipError_t forward_pair(kfac_pinn_ctx* c, const void* xi, int ni, const FwdTarget& Ti,
                        const void* xb, int nb, const FwdTarget& Tb) {
  hipError_t e;
  const Slabs& si = c->si;
  const Slabs& sb = c->sb;
  if ((e = input_slab(Ti.zp, xi, ni, c->d, input_rows_of(c, si, Ti), c->dirs, Ti.z(0), c->ldz[0],
                      c->st)) != hipSuccess ||
      (e = input_slab(Tb.zp, xb, nb, c->d, input_rows_of(c, sb, Tb), c->dirs, Tb.z(0), c->ldz[0],
                      c->st)) != hipSuccess)
    return e;
  for (int l = 0; l < c->L - 1; l++) {
    const LayerLaunch Li = layer_launch(c, si, ni, l, c->L, Ti);
    const LayerLaunch Lb = layer_launch(c, sb, nb, l, c->L, Tb);
    int ti = tm_begin(c, Ti.kc_layer);
    if ((e = fwdlap_pair(Ti.mode, Li.a, Li.nch, &Lb.a, c->st)) != hipSuccess) return e;
    tm_end(c, ti, Li.flops + Lb.flops, Li.bytes + Lb.bytes);
    // the boundary slabs' bias and padding columns are constant (written at creation)
    if ((e = layer_finish(c, Li, Ti)) != hipSuccess) return e;
  }
  return hipSuccess;
}

FwdTarget curvature_target(kfac_pinn_ctx* c, Slabs& s, const void* theta) {
  FwdTarget T;
  T.mode = c->cmode;
  T.zp = c->sp;
  T.zesz = c->esz_s;
  T.theta = theta;
  Slabs* sp = &s;
  T.z = [sp](int l) { return sp->zin_at(l); };
  T.pre = [sp](int l) { return sp->pre_at(l); };
  T.sq = [sp](int l) { return sp->sq[l]; };
  T.u = s.u;
  return T;
}

ResidualTerms residual_terms(const kfac_pinn_ctx* c, const Slabs& s, const void* x) {
  ResidualTerms t;
  if (c->nonlinear && s.has_lap) {
    t.x = x;
    t.mask = c->wts;
    t.d = c->d;
    t.c_x = c->c_x;
    t.c_g = c->c_g;
    t.c_0 = c->c_0;
  }
  return t;
}

// residual, loss[slot] and the seed rows of the output layer
hipError_t residual_and_seed(kfac_pinn_ctx* c, Slabs& s, const void* u, const void* x,
                             const void* y, int n, void* g_last, int slot, int accumulate) {
  hipError_t e;
  const int nb = residual_blocks(n);
  if ((e = residual(c->sp, u, 1, y, n, s.S, time_row_of(c, s), c->c_t, c->c_lap, lap_row_of(s),
                    residual_terms(c, s, x), s.r, s.rf, g_last, c->ldg[c->L - 1], c->partial,
                    c->st)) != hipSuccess)
    return e;
  return finalize_loss(c->partial, nb, 0.5 / (double)n, c->loss, slot, accumulate, c->st);
}

hipError_t residual_loss_only(kfac_pinn_ctx* c, Slabs& s, const void* u, const void* x,
                              const void* y, int n, int slot, int accumulate) {
  hipError_t e;
  const int nb = residual_blocks(n);
  if ((e = residual(c->sp == P_F64 ? P_F64 : P_F32, u, 1, y, n, s.S, time_row_of(c, s), c->c_t,
                    c->c_lap, lap_row_of(s), residual_terms(c, s, x), nullptr, nullptr, nullptr, 1,
                    c->partial, c->st)) != hipSuccess)
    return e;
  return finalize_loss(c->partial, nb, 0.5 / (double)n, c->loss, slot, accumulate, c->st);
}

// Consumer of one layer during the backward sweep.
struct LayerConsumer {
  virtual hipError_t operator()(int l, const void* zin, const void* g) = 0;
};

// Backward sweep from the output seeds (already in g(L-1)).  For each layer l
// (last to first) hands (Z~^(l), g^(l)) to `use`, then forms g^(l-1) by the
// adjoint of the tanh rows at layer l-1.  In recompute mode the forward is
// re-run from x up to layer l whenever layer l's input is needed.
hipError_t backward_sweep(kfac_pinn_ctx* c, Slabs& s, const void* theta, const void* x, int n,
                          LayerConsumer& use) {
  hipError_t e;
  const long R = (long)n * s.S;
  FwdTarget T = curvature_target(c, s, theta);
  for (int l = c->L - 1; l >= 0; l--) {
    if (!s.store && l < c->L - 1) {
      // layer inputs of l (and pre-activations of l-1) from x
      if ((e = forward_run(c, s, x, n, l, T)) != hipSuccess) return e;
    }
    if ((e = use(l, s.zin_at(l), s.g_at(l))) != hipSuccess) return e;
    if (l == 0) break;
    const LayerDesc& ld = c->nd.l[l];
    BwdLayerArgs a{};
    a.N = n;
    a.S = s.S;
    a.nd = s.nd;
    a.has_lap = s.has_lap;
    a.h = ld.h_in;
    a.wts = c->wts;
    a.wts64 = c->wts64;
    a.pre = s.pre_at(l - 1);
    a.ldp = c->ldp[l - 1];
    a.sq = s.sq[l - 1];
    a.g = s.g_at(l - 1);
    a.ldgo = c->ldg[l - 1];
    if (l == c->L - 1) {
      if ((e = bwd_last(c->cmode, a, s.g_at(l), c->ldg[l], wptr(theta, ld.off, c->esz_p),
                        c->st)) != hipSuccess)
        return e;
      continue;
    }
    a.gin = s.g_at(l);
    a.ldgi = c->ldg[l];
    a.w = wptr(c->w_hi, ld.wcm, c->esz_w);
    a.w2 = (c->cmode == M_BF16X3 || c->cmode == M_F16) ? wptr(c->w_lo, ld.wcm, c->esz_w) : nullptr;
    a.ldw = ld.ldk_out;
    a.K = (int)ld.ldk_out;
    const long ts = c->tab_stride;
    a.tab_lb = c->tab;
    a.tab_zv = wptr(c->tab, ts, c->esz_c);
    a.tab_s1 = wptr(c->tab, 2 * ts, c->esz_c);
    const int nch = bwdlap_chunks(c->cmode, n, ld.h_in, s.nd, s.has_lap);
    int ti = tm_begin(c, KC_LAYER_GEMM);
    if ((e = bwdlap_main(c->cmode, a, nch, c->st)) != hipSuccess) return e;
    tm_end(c, ti, 2.0 * R * ld.h_in * ld.h_out,
           (double)R * (ld.h_in + ld.h_out) * c->esz_s + (double)R * ld.h_in * c->esz_c);
    ti = tm_begin(c, KC_ACT);
    if ((e = bwdlap_finish(c->cmode, a, nch, c->st)) != hipSuccess) return e;
    tm_end(c, ti, 0.0, 0.0);
  }
  return hipSuccess;
}

// Factors (EMA) and gradient of one term, from the backward sweep.
struct FactorGrad : LayerConsumer {
  kfac_pinn_ctx* c;
  int term, n, S;
  double beta;
  hipError_t operator()(int l, const void* zin, const void* g) override {
    if (c->defer_products) return hipSuccess;
    hipError_t e;
    const LayerDesc& ld = c->nd.l[l];
    const int K = n * S;
    const int m = c->cmode;
    int sp = 1;
    const double sa = term == 0 ? 1.0 / ((double)n * S) : 1.0 / n;
    const double sbf = 1.0 / n;
    int ti = tm_begin(c, KC_FACTOR_GEMM);
    if ((e = gemm_tn_splitk(m, zin, c->ldz[l], zin, c->ldz[l], ld.h_in + 1, ld.h_in + 1, K,
                            nullptr, nullptr, n, true, c->part, kMaxSplits, &sp, c->st)) !=
        hipSuccess)
      return e;
    tm_end(c, ti, (double)K * (ld.h_in + 1) * (ld.h_in + 2), (double)K * (ld.h_in + 1) * c->esz_s);
    if ((e = reduce_splitk(m, c->part, sp, ld.h_in + 1, ld.h_in + 1, true, c->F[term][0][l],
                           ld.h_in + 1, 1, (1.0 - beta) * sa, beta, c->st)) != hipSuccess)
      return e;
    ti = tm_begin(c, KC_FACTOR_GEMM);
    if ((e = gemm_tn_splitk(m, g, c->ldg[l], g, c->ldg[l], ld.h_out, ld.h_out, K, nullptr,
                            nullptr, n, true, c->part, kMaxSplits, &sp, c->st)) != hipSuccess)
      return e;
    tm_end(c, ti, (double)K * ld.h_out * (ld.h_out + 1), (double)K * ld.h_out * c->esz_s);
    if ((e = reduce_splitk(m, c->part, sp, ld.h_out, ld.h_out, true, c->F[term][1][l], ld.h_out,
                           1, (1.0 - beta) * sbf, beta, c->st)) != hipSuccess)
      return e;
    // gradient: sum_rows (r_n / n) g (x) z~, column-major into theta
    const Slabs& s = term == 0 ? c->si : c->sb;
    ti = tm_begin(c, KC_FACTOR_GEMM);
    if ((e = gemm_tn_splitk(m, g, c->ldg[l], zin, c->ldz[l], ld.h_out, ld.h_in + 1, K, s.r,
                            s.rf, n, false, c->part, kMaxSplits, &sp, c->st, c->wsc)) !=
        hipSuccess)
      return e;
    tm_end(c, ti, 2.0 * K * ld.h_out * (ld.h_in + 1),
           (double)K * (ld.h_out + ld.h_in + 1) * c->esz_s);
    return reduce_splitk(m, c->part, sp, ld.h_out, ld.h_in + 1, false, c->grad + ld.off, 1,
                         ld.h_out, 1.0 / n, term == 0 ? 0.0 : 1.0, c->st);
  }
};

// theta_bar of a general cotangent
struct ThetaBar : LayerConsumer {
  kfac_pinn_ctx* c;
  int n, S;
  double* out;
  hipError_t operator()(int l, const void* zin, const void* g) override {
    const LayerDesc& ld = c->nd.l[l];
    int sp = 1;
    hipError_t e = gemm_tn_splitk(c->cmode, g, c->ldg[l], zin, c->ldz[l], ld.h_out, ld.h_in + 1,
                                  n * S, nullptr, nullptr, n, false, c->part, kMaxSplits, &sp,
                                  c->st);
    if (e != hipSuccess) return e;
    return reduce_splitk(c->cmode, c->part, sp, ld.h_out, ld.h_in + 1, false, out + ld.off, 1,
                         ld.h_out, 1.0, 0.0, c->st);
  }
};

hipError_t prep(kfac_pinn_ctx* c, const void* theta) {
  return prep_weights(c->wp, theta, nullptr, 0.0, c->nd, c->w_hi, c->w_lo, nullptr, 0, c->st);
}

hipError_t curvature_term(kfac_pinn_ctx* c, int term, const void* theta, const void* x,
                          const void* y, int n, double beta) {
  Slabs& s = term == 0 ? c->si : c->sb;
  hipError_t e;
  if (n <= 0) return hipSuccess;
  if ((e = forward_run(c, s, x, n, c->L, curvature_target(c, s, theta))) != hipSuccess) return e;
  if ((e = residual_and_seed(c, s, s.u, x, y, n, s.g_at(c->L - 1), term, 0)) != hipSuccess)
    return e;
  FactorGrad fg;
  fg.c = c; fg.term = term; fg.n = n; fg.S = s.S; fg.beta = beta;
  return backward_sweep(c, s, theta, x, n, fg);
}

// total loss at the parameters in theta_trial (line-search precision) into loss[slot]
// The line-search forward targets: the interior (ping-pong slabs) and the
// boundary (one slab per layer input).
void ls_targets(kfac_pinn_ctx* c, FwdTarget& T, FwdTarget& Tb) {
  T.mode = c->lmode;
  T.zp = c->lp;
  T.zesz = c->esz_l;
  T.theta = c->theta_trial;
  T.z = [c](int l) { return c->ls_z[l & 1]; };
  T.pre = [](int) -> void* { return nullptr; };
  T.sq = [](int) -> void* { return nullptr; };
  T.u = c->ls_u;
  T.kc_layer = KC_LS_LAYER;
  T.full_input = false;
  // The direct-to-LDS products read a row only up to its bias column rounded up to
  // 8 (the rest of the last k-tile reads zeros), so the finishing passes write the
  // bias column and zeros only that far: the rest of each row of the two buffers
  // the layers share is never read.
  T.narrow_pad = c->lmode == M_BF16;
  // a residual with first-order terms reads every derivative row of the output
  T.residual_rows = !c->nonlinear;
  Tb = T;
  Tb.z = [c](int l) { return c->ls_zb[l]; };
  Tb.u = c->ls_ub;
}

// whether a candidate's two point sets take the paired BF16 launches
bool ls_paired(const kfac_pinn_ctx* c, int ni, int nb) {
  return ni > 0 && nb > 0 && c->lmode == M_BF16 && !c->sb.has_lap && c->L >= 2 && !c->nonlinear;
}

hipError_t eval_loss(kfac_pinn_ctx* c, const void* xi, const void* yi, int ni, const void* xb,
                     const void* yb, int nb, int slot) {
  hipError_t e;
  FwdTarget T, Tb;
  ls_targets(c, T, Tb);
  if (ls_paired(c, ni, nb)) {
    if ((e = forward_pair(c, xi, ni, T, xb, nb, Tb)) != hipSuccess) return e;
    const LayerDesc& ld = c->nd.l[c->L - 1];
    return ls_loss(T.mode, T.z(c->L - 1), c->ldz[c->L - 1], ni, time_row_of(c, c->si),
                   lap_row_of(c->si), c->c_t, c->c_lap, yi, Tb.z(c->L - 1), c->ldz[c->L - 1], nb,
                   yb, wptr(T.theta, ld.off, c->esz_p), ld.h_in + 1, c->partial, c->loss + slot,
                   c->st);
  }
  int acc = 0;
  if (ni > 0) {
    if ((e = forward_run(c, c->si, xi, ni, c->L, T)) != hipSuccess) return e;
    if ((e = residual_loss_only(c, c->si, c->ls_u, xi, yi, ni, slot, 0)) != hipSuccess) return e;
    acc = 1;
  }
  if (nb > 0) {
    if ((e = forward_run(c, c->sb, xb, nb, c->L, T)) != hipSuccess) return e;
    if ((e = residual_loss_only(c, c->sb, c->ls_u, xb, yb, nb, slot, acc)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* kfac_pinn_last_error(void) { return g_last_error.c_str(); }

const char* kfac_pinn_status_string(kp_status s) {
  switch (s) {
    case KP_OK: return "ok";
    case KP_ERR_ARG: return "invalid argument";
    case KP_ERR_OOM: return "out of device memory";
    case KP_ERR_HIP: return "HIP error";
    case KP_ERR_NOT_PD: return "damped factor not positive definite";
    case KP_ERR_NONFINITE: return "non-finite loss for every step size";
    case KP_ERR_STATE: return "invalid state";
    case KP_ERR_NOT_CONVERGED: return "eigensolver reached its sweep cap unconverged";
  }
  return "unknown status";
}

int64_t kfac_pinn_num_params(const int32_t* widths, int32_t n_layers) {
  if (!widths || n_layers < 1) return -1;
  int64_t D = 0;
  for (int l = 0; l < n_layers; l++) D += (int64_t)widths[l + 1] * (widths[l] + 1);
  return D;
}

kp_status kfac_pinn_destroy(kfac_pinn_ctx* ctx) {
  if (!ctx) return KP_ERR_ARG;
  if (ctx->ls1.fork) (void)hipEventDestroy(ctx->ls1.fork);
  if (ctx->ls1.join) (void)hipEventDestroy(ctx->ls1.join);
  eig_host_free(ctx->eg);
  if (ctx->eg_streams) {
    for (int k = 1; k < ctx->eg.n; k++) {
      if (ctx->eg.st[k]) {
        (void)hipStreamSynchronize(ctx->eg.st[k]);
        (void)hipStreamDestroy(ctx->eg.st[k]);
      }
      if (ctx->eg.join[k]) (void)hipEventDestroy(ctx->eg.join[k]);
    }
    if (ctx->eg.fork) (void)hipEventDestroy(ctx->eg.fork);
  }
  for (const auto& a : ctx->allocs) (void)hipFree(a.base);
  for (hipEvent_t e : ctx->tm_ev) (void)hipEventDestroy(e);
  delete ctx;
  return KP_OK;
}

static hipError_t ls_lane_alloc(kfac_pinn_ctx* c);

kp_status kfac_pinn_create(const kp_problem* pb, void* stream, kfac_pinn_ctx** out) {
  KP_ARG(pb && out, "null argument");
  *out = nullptr;
  KP_ARG(pb->n_layers >= 1 && pb->n_layers <= kMaxLayers, "n_layers must be in [1, 8]");
  KP_ARG(pb->widths != nullptr, "widths is null");
  for (int l = 0; l <= pb->n_layers; l++)
    KP_ARG(pb->widths[l] >= 1 && pb->widths[l] <= 4096, "widths must be in [1, 4096]");
  KP_ARG(pb->widths[pb->n_layers] == 1, "the network output must be scalar (widths[L] == 1)");
  KP_ARG(pb->widths[0] <= 1024, "at most 1024 inputs");
  KP_ARG(pb->precision >= KP_F64 && pb->precision <= KP_MIXED_F16, "unknown precision");
  KP_ARG(pb->max_interior >= 0 && pb->max_boundary >= 0, "negative capacity");
  KP_ARG(pb->time_coord >= -1 && pb->time_coord < pb->widths[0], "time_coord out of range");
  KP_ARG(std::isfinite(pb->coef_xgrad) && std::isfinite(pb->coef_gradsq) &&
             std::isfinite(pb->coef_const),
         "first-order residual coefficients must be finite");
  KP_ARG(!(pb->op_coef && (pb->coef_xgrad != 0.0 || pb->coef_gradsq != 0.0)),
         "first-order residual terms need the mask form of the operator (no op_coef)");
  if (pb->op_coef) {
    const int d = pb->widths[0];
    KP_ARG(!pb->lap_mask, "give either lap_mask or op_coef");
    double mx = 0.0;
    for (long e = 0; e < (long)d * d; e++) {
      KP_ARG(std::isfinite(pb->op_coef[e]), "op_coef must be finite");
      mx = std::max(mx, std::fabs(pb->op_coef[e]));
    }
    for (int i = 0; i < d; i++)
      for (int j = 0; j < i; j++)
        KP_ARG(std::fabs(pb->op_coef[(long)i * d + j] - pb->op_coef[(long)j * d + i]) <= 1e-12 * mx,
               "op_coef must be symmetric");
    if (pb->time_coord >= 0 && pb->coef_time != 0.0)
      for (int i = 0; i < d; i++)
        KP_ARG(pb->op_coef[(long)pb->time_coord * d + i] == 0.0,
               "op_coef: the time coordinate's row and column must be zero");
  }

  kfac_pinn_ctx* c = new kfac_pinn_ctx();
  if (const char* gk = getenv("KFAC_PINN_GUARD_KB")) {
    const long kb = atol(gk);
    if (kb > 0) c->guard = (size_t)std::min(kb, 1L << 20) * 1024;
  }
  c->L = pb->n_layers;
  c->w.assign(pb->widths, pb->widths + pb->n_layers + 1);
  c->d = c->w[0];
  c->time_coord = pb->time_coord;
  c->c_t = pb->coef_time;
  c->c_lap = pb->coef_lap;
  c->c_x = pb->coef_xgrad;
  c->c_g = pb->coef_gradsq;
  c->c_0 = pb->coef_const;
  c->nonlinear = c->c_x != 0.0 || c->c_g != 0.0 || c->c_0 != 0.0;
  c->precision = pb->precision;
  if (pb->precision == KP_F64) {
    c->pp = c->sp = c->lp = c->wp = P_F64;
    c->cmode = c->lmode = M_F64;
    c->esz_p = c->esz_s = c->esz_l = c->esz_c = c->esz_w = 8;
  } else if (pb->precision == KP_F32) {
    c->pp = c->sp = c->lp = c->wp = P_F32;
    c->cmode = c->lmode = M_F32;
    c->esz_p = c->esz_s = c->esz_l = c->esz_c = c->esz_w = 4;
  } else {   // mixed: FP32 slabs with BF16x3 or FP16 products for the curvature pass, BF16 line search
    c->pp = c->sp = P_F32;
    c->lp = P_BF16;
    c->wp = pb->precision == KP_MIXED_F16 ? P_F16 : P_BF16;
    c->cmode = pb->precision == KP_MIXED_F16 ? M_F16 : M_BF16X3;
    c->lmode = M_BF16;
    c->esz_p = c->esz_s = c->esz_c = 4;
    c->esz_l = c->esz_w = 2;
  }
  c->max_i = pb->max_interior;
  c->max_b = pb->max_boundary;
  c->ws_limit = pb->workspace_limit_bytes;
  c->st = (hipStream_t)stream;
  c->D = kfac_pinn_num_params(pb->widths, pb->n_layers);

  // layer geometry
  c->nd.L = c->L;
  long woff = 0, toff = 0;
  for (int l = 0; l < c->L; l++) {
    const int hi = c->w[l], ho = c->w[l + 1];
    LayerDesc& ld = c->nd.l[l];
    ld.h_in = hi;
    ld.h_out = ho;
    ld.off = toff;
    ld.ldk_in = kp_roundup(hi + 1, 64);
    ld.ldk_out = kp_roundup(ho, 8);
    ld.wrm = woff;
    woff += (long)ho * ld.ldk_in;
    ld.wcm = woff;
    woff += (long)hi * ld.ldk_out;
    c->off.push_back(toff);
    c->ldz.push_back(ld.ldk_in);
    c->ldp.push_back(kp_roundup(ho, 8));
    c->ldg.push_back(ld.ldk_out);
    toff += (long)ho * (hi + 1);
    c->ldz_max = std::max(c->ldz_max, (long)ld.ldk_in);
    c->ldp_max = std::max(c->ldp_max, kp_roundup(std::max(hi, ho), 8));
  }
  c->si.S = c->d + 2;
  c->si.nd = c->d;
  c->si.has_lap = 1;
  c->si.cap = c->max_i;
  c->sb.S = 1;
  c->sb.nd = 0;
  c->sb.has_lap = 0;
  c->sb.cap = c->max_b;
  c->si.store = !(c->ws_limit > 0 && slab_bytes(c, c->si, true) > c->ws_limit);
  c->sb.store = true;

  hipError_t e = hipSuccess;
#define ALLOC(ptr, bytes)                                          \
  if ((e = dmalloc(c, (void**)&(ptr), (bytes))) != hipSuccess) {  \
    kp_set_last_error(hipGetErrorString(e), __FILE__, __LINE__);   \
    kfac_pinn_destroy(c);                                          \
    return e == hipErrorOutOfMemory ? KP_ERR_OOM : KP_ERR_HIP;    \
  }
  // Second-order part of the operator: sum_k w_k d^2/dv_k^2 along orthonormal
  // directions v_k.  A mask gives v_k = e_k and w_k in {0, 1}; a coefficient
  // matrix C gives its eigenvectors and eigenvalues (Appendix C.3's operator
  // sum_ij C_ij d_i d_j, diagonal in that basis).
  {
    std::vector<double> V, w;
    if (pb->op_coef) {
      eig_sym_host(c->d, pb->op_coef, V, w);
      bool ident = true;
      for (int i = 0; i < c->d && ident; i++)
        for (int k = 0; k < c->d; k++)
          if (V[(long)i * c->d + k] != (i == k ? 1.0 : 0.0)) { ident = false; break; }
      if (!ident) {
        std::vector<double> rows((size_t)c->d * c->d);   // row k = v_k
        for (int i = 0; i < c->d; i++)
          for (int k = 0; k < c->d; k++) rows[(size_t)k * c->d + i] = V[(size_t)i * c->d + k];
        ALLOC(c->dirs, sizeof(double) * rows.size());
        if ((e = hipMemcpy(c->dirs, rows.data(), sizeof(double) * rows.size(),
                           hipMemcpyHostToDevice)) != hipSuccess) {
          kfac_pinn_destroy(c);
          return KP_ERR_HIP;
        }
      }
    } else {
      w.resize(c->d);
      for (int i = 0; i < c->d; i++) w[i] = (!pb->lap_mask || pb->lap_mask[i]) ? 1.0 : 0.0;
    }
    std::vector<float> wf(kp_roundup(c->d, 4), 0.0f);
    std::vector<double> wd(kp_roundup(c->d, 4), 0.0);
    for (int i = 0; i < c->d; i++) {
      wf[i] = (float)w[i];
      wd[i] = w[i];
    }
    ALLOC(c->wts, sizeof(float) * wf.size());
    ALLOC(c->wts64, sizeof(double) * wd.size());
    if ((e = hipMemcpy(c->wts, wf.data(), sizeof(float) * wf.size(), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(c->wts64, wd.data(), sizeof(double) * wd.size(),
                       hipMemcpyHostToDevice)) != hipSuccess) {
      kfac_pinn_destroy(c);
      return KP_ERR_HIP;
    }
  }
  c->w_bytes = (size_t)woff * c->esz_w;
  ALLOC(c->w_hi, c->w_bytes);
  if (c->wp == P_BF16 || c->wp == P_F16) ALLOC(c->w_lo, (size_t)woff * c->esz_w);
  ALLOC(c->theta_trial, (size_t)c->D * c->esz_p);
  if ((e = alloc_slabs(c, c->si)) != hipSuccess || (e = alloc_slabs(c, c->sb)) != hipSuccess) {
    kp_set_last_error(hipGetErrorString(e), __FILE__, __LINE__);
    kfac_pinn_destroy(c);
    return e == hipErrorOutOfMemory ? KP_ERR_OOM : KP_ERR_HIP;
  }
  const size_t Rmax = std::max((size_t)c->max_i * c->si.S, (size_t)c->max_b);
  ALLOC(c->ls_z[0], Rmax * c->ldz_max * c->esz_l);
  ALLOC(c->ls_z[1], Rmax * c->ldz_max * c->esz_l);
  ALLOC(c->ls_u, Rmax * c->esz_c);
  if (c->lmode == M_BF16 && c->max_b > 0) {
    const size_t Rb = (size_t)c->max_b * c->sb.S;
    for (int l = 0; l < c->L; l++) ALLOC(c->ls_zb[l], Rb * c->ldz[l] * c->esz_l);
    // the zero fills run on the null stream: finish them before the padding
    // kernels on the context's stream, which may be a non-blocking one
    if ((e = hipDeviceSynchronize()) != hipSuccess) {
      kp_set_last_error(hipGetErrorString(e), __FILE__, __LINE__);
      kfac_pinn_destroy(c);
      return KP_ERR_HIP;
    }
    for (int l = 1; l < c->L; l++) {
      FwdLayerArgs a{};
      a.N = c->max_b;
      a.S = 1;
      a.h_out = c->w[l];
      a.z = c->ls_zb[l];
      a.ldzo = c->ldz[l];
      if ((e = fwdlap_finish(c->lmode, a, 1, c->st)) != hipSuccess ||
          (e = hipStreamSynchronize(c->st)) != hipSuccess) {
        kp_set_last_error(hipGetErrorString(e), __FILE__, __LINE__);
        kfac_pinn_destroy(c);
        return KP_ERR_HIP;
      }
    }
    ALLOC(c->ls_ub, Rb * c->esz_c);
  }
  {
    int hmax = 1;
    for (int l = 1; l < c->L; l++) hmax = std::max(hmax, c->w[l]);
    c->tab_stride = ((long)std::max(c->max_i, 1) * hmax + 3) & ~3L;   // 16-byte planes
    ALLOC(c->tab, (size_t)c->tab_stride * (2 + kMaxChunks) * c->esz_c);
  }
  c->partial_n = std::max(residual_blocks(std::max(c->max_i, c->max_b)),
                          ls_loss_blocks(c->max_i, c->max_b));
  ALLOC(c->partial, sizeof(double) * c->partial_n);
  ALLOC(c->loss, sizeof(double) * (2 + kMaxCand + 2));
  for (int t = 0; t < 2; t++)
    for (int sd = 0; sd < 2; sd++) {
      c->F[t][sd].resize(c->L);
      for (int l = 0; l < c->L; l++) {
        const long n = sd == 0 ? c->w[l] + 1 : c->w[l + 1];
        ALLOC(c->F[t][sd][l], sizeof(double) * n * n);
      }
    }
  {
    long mn = 0;   // largest product output: A (h_in+1)^2, B h_out^2, gradient h_out (h_in+1)
    for (int l = 0; l < c->L; l++) {
      const long a = c->w[l] + 1, b = c->w[l + 1];
      mn = std::max(mn, std::max(a * a, std::max(b * b, a * b)));
    }
    ALLOC(c->part, (size_t)kMaxSplits * mn * c->esz_c);
    ALLOC(c->wsc, 2 * sizeof(float));
  }
  ALLOC(c->grad, sizeof(double) * c->D);
  ALLOC(c->Delta, sizeof(double) * c->D);
  ALLOC(c->dhat, c->esz_p * c->D);
  ALLOC(c->delta, c->esz_p * c->D);
  ALLOC(c->ctl, sizeof(int) * 128);
  {
    c->jv_ld = std::max(1, std::max(c->max_i, c->max_b));
    ALLOC(c->jv, sizeof(double) * 4 * c->jv_ld);
    int ntj = 1;
    for (int l = 0; l < c->L; l++) ntj = std::max(ntj, jvp_tiles(c->w[l + 1]));
    const size_t Rmax = std::max((size_t)c->max_i * c->si.S, (size_t)c->max_b);
    ALLOC(c->jvp_part, 2 * (size_t)ntj * std::max(Rmax, (size_t)1) * c->esz_s);
  }
  ALLOC(c->qbuf, sizeof(double) * (size_t)(c->d + 1) * c->w[1]);

  // eigenproblems: layer l side A (h_in+1) and side B (h_out)
  for (int l = 0; l < c->L; l++)
    for (int sd = 0; sd < 2; sd++) {
      EigProblem p{};
      p.n = sd == 0 ? c->w[l] + 1 : c->w[l + 1];
      p.n_pad = (int)kp_roundup(p.n, 64);
      p.f1 = c->F[0][sd][l];
      p.f2 = c->F[1][sd][l];
      const size_t np2 = (size_t)p.n_pad * p.n_pad * sizeof(double);
      ALLOC(p.M1, np2);
      ALLOC(p.M2, np2);
      ALLOC(p.Lb, np2);
      ALLOC(p.Li, np2);
      ALLOC(p.C[0], np2);
      ALLOC(p.C[1], np2);
      ALLOC(p.P[0], np2);
      ALLOC(p.P[1], np2);
      ALLOC(p.V, (size_t)(p.n_pad / 64) * 64 * 64 * sizeof(double));
      ALLOC(p.pflag, (size_t)(p.n_pad / 64 + 1) * sizeof(int));
      ALLOC(p.dmax, sizeof(double));
      ALLOC(p.Pout, (size_t)p.n * p.n * sizeof(double));
      ALLOC(p.eout, (size_t)p.n * sizeof(double));
      p.status = c->ctl;
      c->probs.push_back(p);
    }
  ALLOC(c->probs_dev, sizeof(EigProblem) * c->probs.size());
  if ((e = hipMemcpy(c->probs_dev, c->probs.data(), sizeof(EigProblem) * c->probs.size(),
                     hipMemcpyHostToDevice)) != hipSuccess) {
    kfac_pinn_destroy(c);
    return KP_ERR_HIP;
  }
  {
    std::vector<int> ids(c->probs.size());
    eig_groups_plan(c->probs.data(), (int)c->probs.size(), kEigGroups, ids.data(), c->eg);
    int* ids_dev = nullptr;
    ALLOC(ids_dev, sizeof(int) * ids.size());
    if ((e = hipMemcpy(ids_dev, ids.data(), sizeof(int) * ids.size(), hipMemcpyHostToDevice)) !=
        hipSuccess) {
      kfac_pinn_destroy(c);
      return KP_ERR_HIP;
    }
    c->eg.ids = ids_dev;
    if ((e = eig_host_sync(c->eg, ids.data(), (int)ids.size())) != hipSuccess) {
      kfac_pinn_destroy(c);
      return KP_ERR_HIP;
    }
  }
  {
    std::vector<KronApply> ka(c->L);
    long tstride = 0;
    for (int l = 0; l < c->L; l++) {
      ka[l].nA = c->w[l] + 1;
      ka[l].nB = c->w[l + 1];
      ka[l].off = c->off[l];
      ka[l].PA = c->probs[2 * l].Pout;
      ka[l].a = c->probs[2 * l].eout;
      ka[l].PB = c->probs[2 * l + 1].Pout;
      ka[l].b = c->probs[2 * l + 1].eout;
      tstride = std::max(tstride, 2L * ka[l].nA * ka[l].nB);
    }
    double* ktmp = nullptr;
    ALLOC(ktmp, sizeof(double) * tstride * c->L);
    std::vector<G64> h(4 * c->L);
    kron_apply_descs(ka.data(), c->L, c->grad, c->Delta, ktmp, tstride, h.data(), &c->k_mmax,
                     &c->k_nmax);
    ALLOC(c->kdesc, sizeof(G64) * h.size());
    if ((e = hipMemcpy(c->kdesc, h.data(), sizeof(G64) * h.size(), hipMemcpyHostToDevice)) !=
        hipSuccess) {
      kfac_pinn_destroy(c);
      return KP_ERR_HIP;
    }
  }
#undef ALLOC
  // Algorithm 1, step 0: identity factors, zero momentum
  for (int t = 0; t < 2; t++)
    for (int sd = 0; sd < 2; sd++)
      for (int l = 0; l < c->L; l++) {
        const long n = sd == 0 ? c->w[l] + 1 : c->w[l + 1];
        if ((e = ema_fill(c->F[t][sd][l], n * n, (int)n, 1, nullptr)) != hipSuccess) {
          kfac_pinn_destroy(c);
          return KP_ERR_HIP;
        }
      }
  if ((e = hipDeviceSynchronize()) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->ls1.fork, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->ls1.join, hipEventDisableTiming)) != hipSuccess ||
      (e = ls_lane_alloc(c)) != hipSuccess) {
    kp_set_last_error(hipGetErrorString(e), __FILE__, __LINE__);
    kfac_pinn_destroy(c);
    return e == hipErrorOutOfMemory ? KP_ERR_OOM : KP_ERR_HIP;
  }
  *out = c;
  return KP_OK;
}

kp_status kfac_pinn_reset_state(kfac_pinn_ctx* c, int32_t init_identity) {
  KP_ARG(c, "null context");
  for (int t = 0; t < 2; t++)
    for (int sd = 0; sd < 2; sd++)
      for (int l = 0; l < c->L; l++) {
        const long n = sd == 0 ? c->w[l] + 1 : c->w[l + 1];
        KP_TRY(ema_fill(c->F[t][sd][l], n * n, (int)n, init_identity ? 1 : 0, c->st));
      }
  KP_TRY(zero_fill(c->delta, c->esz_p * c->D, c->st));
  KP_TRY(zero_fill(c->ctl, sizeof(int) * 8, c->st));
  return KP_OK;
}

kp_status kfac_pinn_sample(kfac_pinn_ctx* c, const kp_sampler* s, int64_t step, void* x_int,
                           void* y_int, void* x_bnd, void* y_bnd) {
  KP_ARG(c && s, "null argument");
  KP_ARG(s->n_interior >= 0 && s->n_boundary >= 0 && s->n_initial >= 0, "negative count");
  KP_ARG(s->face_lo >= 0 && s->face_lo < c->d, "face_lo out of range");
  KP_ARG(s->target_kind >= 0 && s->target_kind <= 2, "unknown target kind");
  KP_ARG(s->target_kind != 1 || c->d >= 2, "target kind 1 needs d >= 2");
  KP_ARG(s->n_interior == 0 || (x_int && y_int), "interior buffers are null");
  KP_ARG(s->n_boundary + s->n_initial == 0 || (x_bnd && y_bnd), "boundary buffers are null");
  KP_ARG(step >= 0, "negative step");
  SamplerDesc sd;
  sd.seed_i = s->seed_interior;
  sd.seed_b = s->seed_boundary;
  sd.seed_0 = s->seed_initial;
  sd.n_i = s->n_interior;
  sd.n_b = s->n_boundary;
  sd.n_0 = s->n_initial;
  sd.d = c->d;
  sd.face_lo = s->face_lo;
  sd.kind = s->target_kind;
  sd.scale = s->scale;
  sd.kappa = s->kappa;
  sd.step = (long)step;
  KP_TRY(sample(c->pp, sd, x_int, y_int, x_bnd, y_bnd, c->st));
  return KP_OK;
}

kp_status kfac_pinn_forward_laplacian(kfac_pinn_ctx* c, const void* theta, const void* x,
                                      int32_t n, void* u_out, void* grad_out, void* lap_out) {
  KP_ARG(c && theta && x, "null argument");
  KP_ARG(n >= 0 && n <= c->max_i, "n exceeds max_interior");
  if (n == 0) return KP_OK;
  KP_TRY(prep(c, theta));
  KP_TRY(forward_run(c, c->si, x, n, c->L, curvature_target(c, c->si, theta)));
  KP_TRY(extract_outputs(c->pp, c->si.u, 1, n, c->si.S, c->d, c->si.S - 1, c->dirs, u_out,
                         grad_out,
                         lap_out, c->st));
  return KP_OK;
}

kp_status kfac_pinn_forward_laplacian_vjp(kfac_pinn_ctx* c, const void* theta, const void* x,
                                          int32_t n, const void* u_bar, const void* grad_bar,
                                          const void* lap_bar, double* theta_bar, void* x_bar) {
  KP_ARG(c && theta && x && theta_bar, "null argument");
  KP_ARG(n >= 0 && n <= c->max_i, "n exceeds max_interior");
  if (n == 0) {
    KP_TRY(zero_fill(theta_bar, sizeof(double) * c->D, c->st));
    return KP_OK;
  }
  Slabs& s = c->si;
  KP_TRY(prep(c, theta));
  // stored mode: slabs of this (theta, x); recompute mode: the last hidden layer's
  // inputs and pre-activations for the first backward step
  KP_TRY(forward_run(c, s, x, n, c->L, curvature_target(c, s, theta)));
  KP_TRY(seed_rows(c->sp, u_bar, grad_bar, lap_bar, n, s.S, c->d, s.S - 1, c->dirs,
                   s.g_at(c->L - 1),
                   c->ldg[c->L - 1], c->st));
  ThetaBar tb;
  tb.c = c;
  tb.n = n;
  tb.S = s.S;
  tb.out = theta_bar;
  KP_TRY(backward_sweep(c, s, theta, x, n, tb));
  if (x_bar)
    KP_TRY(input_vjp(c->sp, theta, c->w[1], c->d, s.g_at(0), c->ldg[0], n, s.S, x_bar, c->st));
  return KP_OK;
}

static kp_status check_batch(kfac_pinn_ctx* c, const void* xi, const void* yi, int ni,
                             const void* xb, const void* yb, int nb) {
  KP_ARG(ni >= 0 && ni <= c->max_i, "n_int exceeds max_interior");
  KP_ARG(nb >= 0 && nb <= c->max_b, "n_bnd exceeds max_boundary");
  KP_ARG(ni == 0 || (xi && yi), "interior buffers are null");
  KP_ARG(nb == 0 || (xb && yb), "boundary buffers are null");
  KP_ARG(ni + nb > 0, "empty batch");
  return KP_OK;
}

// EMA of one term's factors toward zero (a term without points contributes 0)
static hipError_t decay_term(kfac_pinn_ctx* c, int term, double beta) {
  for (int sd = 0; sd < 2; sd++)
    for (int l = 0; l < c->L; l++) {
      const int n = sd == 0 ? c->w[l] + 1 : c->w[l + 1];
      hipError_t e = reduce_splitk(c->cmode, c->part, 0, n, n, true, c->F[term][sd][l], n, 1, 0.0,
                                   beta, c->st);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

static kp_status factors_impl(kfac_pinn_ctx* c, const void* theta, const void* xi, const void* yi,
                              int ni, const void* xb, const void* yb, int nb, double beta) {
  KP_TRY(prep(c, theta));
  KP_TRY(zero_fill(c->grad, sizeof(double) * c->D, c->st));
  KP_TRY(zero_fill(c->loss, sizeof(double) * 2, c->st));
  c->last_n[0] = ni;
  c->last_n[1] = nb;
  // interior term first: it overwrites the gradient, the boundary term adds to it
  if (ni > 0) KP_TRY(curvature_term(c, 0, theta, xi, yi, ni, beta));
  else KP_TRY(decay_term(c, 0, beta));
  if (nb > 0) KP_TRY(curvature_term(c, 1, theta, xb, yb, nb, beta));
  else KP_TRY(decay_term(c, 1, beta));
  return KP_OK;
}

kp_status kfac_pinn_factors(kfac_pinn_ctx* c, const void* theta, const void* xi, const void* yi,
                            int32_t ni, const void* xb, const void* yb, int32_t nb, double beta,
                            double* grad_out, double* loss_out) {
  KP_ARG(c && theta, "null argument");
  KP_ARG(beta >= 0.0 && beta < 1.0, "beta must be in [0, 1)");
  kp_status s = check_batch(c, xi, yi, ni, xb, yb, nb);
  if (s != KP_OK) return s;
  s = factors_impl(c, theta, xi, yi, ni, xb, yb, nb, beta);
  if (s != KP_OK) return s;
  if (grad_out)
    KP_TRY(hipMemcpyAsync(grad_out, c->grad, sizeof(double) * c->D, hipMemcpyDeviceToDevice,
                          c->st));
  if (loss_out)
    KP_TRY(hipMemcpyAsync(loss_out, c->loss, sizeof(double) * 2, hipMemcpyDeviceToDevice, c->st));
  return KP_OK;
}

// side streams of default priority for the concurrent Jacobi groups (the first
// one also carries line-search lane 1)
static hipError_t side_streams(kfac_pinn_ctx* c) {
  if (c->eg_streams || c->eg.n < 2) return hipSuccess;
  c->eg_streams = true;
  for (int k = 1; k < c->eg.n; k++) {
    if (hipError_t e = hipStreamCreateWithFlags(&c->eg.st[k], hipStreamNonBlocking)) return e;
    if (hipError_t e = hipEventCreateWithFlags(&c->eg.join[k], hipEventDisableTiming)) return e;
  }
  return hipEventCreateWithFlags(&c->eg.fork, hipEventDisableTiming);
}

// Buffers of line-search lane 1, sized as lane 0's (the context's own); its
// stream is the first side stream, attached when a step uses the lane.
static hipError_t ls_lane_alloc(kfac_pinn_ctx* c) {
  kfac_pinn_ctx::LsLane& x = c->ls1;
  if (x.ready) return hipSuccess;
  hipError_t e;
  const size_t Rmax = std::max((size_t)c->max_i * c->si.S, (size_t)c->max_b);
  if ((e = dmalloc(c, &x.theta_trial, (size_t)c->D * c->esz_p)) != hipSuccess ||
      (e = dmalloc(c, &x.w_hi, c->w_bytes)) != hipSuccess ||
      (e = dmalloc(c, &x.ls_z[0], Rmax * c->ldz_max * c->esz_l)) != hipSuccess ||
      (e = dmalloc(c, &x.ls_z[1], Rmax * c->ldz_max * c->esz_l)) != hipSuccess ||
      (e = dmalloc(c, &x.ls_u, Rmax * c->esz_c)) != hipSuccess ||
      (e = dmalloc(c, &x.tab, (size_t)c->tab_stride * (2 + kMaxChunks) * c->esz_c)) != hipSuccess ||
      (e = dmalloc(c, (void**)&x.partial, sizeof(double) * c->partial_n)) != hipSuccess ||
      (e = dmalloc(c, &x.qbuf, sizeof(double) * (size_t)(c->d + 1) * c->w[1])) != hipSuccess)
    return e;
  const size_t Rb = (size_t)c->max_b * c->sb.S;
  if (c->ls_zb[0]) {
    for (int l = 0; l < c->L; l++)
      if ((e = dmalloc(c, &x.ls_zb[l], Rb * c->ldz[l] * c->esz_l)) != hipSuccess) return e;
    if ((e = dmalloc(c, &x.ls_ub, Rb * c->esz_c)) != hipSuccess) return e;
  }
  // the zero fills of dmalloc run on the null stream, which a non-blocking stream
  // does not wait for: finish them before the padding kernels
  if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
  if (c->ls_zb[0]) {   // boundary slabs with their constant bias and padding columns
    for (int l = 1; l < c->L; l++) {
      FwdLayerArgs a{};
      a.N = c->max_b;
      a.S = 1;
      a.h_out = c->w[l];
      a.z = x.ls_zb[l];
      a.ldzo = c->ldz[l];
      if ((e = fwdlap_finish(c->lmode, a, 1, c->st)) != hipSuccess) return e;
    }
    if ((e = hipStreamSynchronize(c->st)) != hipSuccess) return e;
  }
  x.ready = true;
  return hipSuccess;
}

static hipError_t ls_lane_free(kfac_pinn_ctx* c) {
  kfac_pinn_ctx::LsLane& x = c->ls1;
  if (!x.ready) return hipSuccess;
  if (hipError_t e = hipDeviceSynchronize()) return e;
  std::vector<void*> bufs = {x.theta_trial, x.w_hi, x.ls_z[0], x.ls_z[1], x.ls_u, x.ls_ub,
                             x.tab, x.partial, x.qbuf};
  for (int l = 0; l < kMaxLayers; l++) bufs.push_back(x.ls_zb[l]);
  for (void* b : bufs) {
    if (!b) continue;
    dfree(c, b);
  }
  hipStream_t st = x.st;
  hipEvent_t f = x.fork, j = x.join;
  x = kfac_pinn_ctx::LsLane{};
  x.st = st;
  x.fork = f;
  x.join = j;
  return hipSuccess;
}

// Exchanges the context's stream and line-search buffers with lane 1's: the
// line-search helpers then enqueue a candidate on lane 1.
static void ls_lane_swap(kfac_pinn_ctx* c) {
  kfac_pinn_ctx::LsLane& x = c->ls1;
  std::swap(c->st, x.st);
  std::swap(c->theta_trial, x.theta_trial);
  std::swap(c->w_hi, x.w_hi);
  std::swap(c->ls_z[0], x.ls_z[0]);
  std::swap(c->ls_z[1], x.ls_z[1]);
  std::swap(c->ls_u, x.ls_u);
  for (int l = 0; l < kMaxLayers; l++) std::swap(c->ls_zb[l], x.ls_zb[l]);
  std::swap(c->ls_ub, x.ls_ub);
  std::swap(c->tab, x.tab);
  std::swap(c->partial, x.partial);
  std::swap(c->qbuf, x.qbuf);
}

static hipError_t eig_all(kfac_pinn_ctx* c, double lambda) {
  if (hipError_t e = side_streams(c)) return e;
  return kron_eig_batched(c->probs.data(), (int)c->probs.size(), lambda, c->probs_dev, c->ctl,
                          c->ctl + 8, c->ctl + 2, kEigRefresh, c->max_sweeps, c->eg, c->st);
}

kp_status kfac_pinn_invert(kfac_pinn_ctx* c, double lambda) {
  KP_ARG(c, "null context");
  KP_ARG(lambda >= 0.0 && isfinite(lambda), "lambda must be finite and >= 0");
  KP_TRY(eig_all(c, lambda));
  return KP_OK;
}

kp_status kfac_pinn_precondition_layer_noalloc(int32_t nA, int32_t nB, const double* PA,
                                               const double* a, const double* PB, const double* b,
                                               const double* grad, double* delta, void* stream) {
  KP_ARG(PA && a && PB && b && grad && delta, "null argument");
  KP_ARG(nA >= 1 && nB >= 1, "nA and nB must be positive");
  KP_ARG((long)nA * nB <= kKronScratchElems,
         "nA * nB exceeds the static scratch (1048576 elements per product)");
  KronApply k{};
  k.nA = nA;
  k.nB = nB;
  k.PA = PA;
  k.a = a;
  k.PB = PB;
  k.b = b;
  KP_TRY(kron_apply_noalloc(k, grad, delta, (hipStream_t)stream));
  return KP_OK;
}

kp_status kfac_pinn_layer_gramian(kfac_pinn_ctx* c, int32_t layer, int32_t term, double* out,
                                  double* work) {
  KP_ARG(c && out && work, "null argument");
  KP_ARG(layer >= 0 && layer < c->L && (term == 0 || term == 1), "index out of range");
  const Slabs& s = term == 0 ? c->si : c->sb;
  KP_ARG(s.store, "the exact Gramian needs the stored slabs (no workspace limit)");
  const int n = c->last_n[term];
  KP_ARG(n > 0, "no curvature pass with points of this term yet");
  const LayerDesc& ld = c->nd.l[layer];
  const long p = (long)ld.h_out * (ld.h_in + 1);
  KP_ARG(p <= kMaxGramianParams, "layer too large for the exact Gramian (more than 16384 parameters)");
  KP_TRY(layer_gramian(c->sp == P_F64 ? P_F64 : P_F32, s.zin_at(layer), c->ldz[layer],
                       s.g_at(layer), c->ldg[layer], n, s.S, ld.h_in + 1, ld.h_out, work, out,
                       c->st));
  return KP_OK;
}

kp_status kfac_pinn_set_max_sweeps(kfac_pinn_ctx* c, int32_t max_sweeps) {
  KP_ARG(c, "null context");
  KP_ARG(max_sweeps >= 1 && max_sweeps <= 64, "max_sweeps must be in [1, 64]");
  c->max_sweeps = max_sweeps;
  return KP_OK;
}

kp_status kfac_pinn_set_sweep_wait(kfac_pinn_ctx* c, int32_t enabled) {
  KP_ARG(c, "null context");
  KP_ARG(enabled == 0 || enabled == 1, "enabled must be 0 or 1");
  c->eg.host_wait = enabled == 1;
  return KP_OK;
}

kp_status kfac_pinn_check_guards(kfac_pinn_ctx* c, int64_t* bad_bytes, int64_t* buffers) {
  KP_ARG(c && bad_bytes && buffers, "null argument");
  *bad_bytes = 0;
  *buffers = 0;
  if (c->guard == 0) return KP_OK;
  KP_TRY(hipDeviceSynchronize());
  std::vector<unsigned char> h(c->guard);
  for (const auto& a : c->allocs) {
    const char* regions[2] = {(const char*)a.base, (const char*)a.user + a.bytes};
    for (const char* r : regions) {
      KP_TRY(hipMemcpy(h.data(), r, c->guard, hipMemcpyDeviceToHost));
      for (unsigned char v : h) *bad_bytes += v != kGuardByte;
    }
    *buffers += 1;
  }
  return KP_OK;
}

kp_status kfac_pinn_precondition(kfac_pinn_ctx* c, const double* grad_in, double* delta_out) {
  KP_ARG(c && grad_in && delta_out, "null argument");
  if (grad_in != c->grad)
    KP_TRY(hipMemcpyAsync(c->grad, grad_in, sizeof(double) * c->D, hipMemcpyDeviceToDevice, c->st));
  KP_TRY(kron_apply_batched(c->kdesc, c->L, c->k_mmax, c->k_nmax, c->st));
  KP_TRY(hipMemcpyAsync(delta_out, c->Delta, sizeof(double) * c->D, hipMemcpyDeviceToDevice,
                        c->st));
  return KP_OK;
}

// A step in three parts: the factors and gradient (head), the inversion, and the
// direction, line search and update (tail).  A batch runs the heads of all its
// instances, one inversion over all of their factors, then the tails.
static kp_status step_head(kfac_pinn_ctx* c, void* theta, const void* xi, const void* yi,
                           int32_t ni, const void* xb, const void* yb, int32_t nb,
                           const kp_hparams* hp) {
  KP_ARG(c && theta && hp, "null argument");
  KP_ARG(hp->beta >= 0.0 && hp->beta < 1.0, "beta must be in [0, 1)");
  KP_ARG(hp->lambda >= 0.0 && isfinite(hp->lambda), "lambda must be finite and >= 0");
  KP_ARG(isfinite(hp->momentum), "momentum must be finite");
  KP_ARG(hp->lr_mode >= 0 && hp->lr_mode <= 2, "lr_mode must be 0, 1 or 2");
  KP_ARG(hp->lr_mode != 2 || c->si.store,
         "KFAC* (lr_mode 2) needs the stored interior slabs (no workspace limit)");
  if (hp->lr_mode == 1) {
    KP_ARG(hp->grid_max_exp >= hp->grid_min_exp, "empty line-search grid");
    KP_ARG(hp->grid_max_exp - hp->grid_min_exp + 1 <= kMaxCand,
           "at most 64 line-search candidates");
    KP_ARG(hp->grid_max_exp <= 60 && hp->grid_min_exp >= -1000, "grid exponents out of range");
  } else {
    KP_ARG(hp->lr >= 0.0 && isfinite(hp->lr), "lr must be finite and >= 0");
  }
  kp_status s = check_batch(c, xi, yi, ni, xb, yb, nb);
  if (s != KP_OK) return s;
  // 1-2) factors, EMA, losses and gradient at theta_t
  return factors_impl(c, theta, xi, yi, ni, xb, yb, nb, hp->beta);
}

// KFAC* (Section 3.4): the residuals' Jacobian-vector products along Delta and
// delta_{t-1} from the slabs the curvature pass stored (layer by layer, interior
// and boundary), then the 2 x 2 quadratic model and the update.
static kp_status kstar_tail(kfac_pinn_ctx* c, void* theta, int32_t ni, int32_t nb,
                            const kp_hparams* hp, kp_step_info* info) {
  const Prec sp = c->sp == P_F64 ? P_F64 : P_F32;   // slab type of the curvature pass
  for (int term = 0; term < 2; term++) {
    const Slabs& s = term == 0 ? c->si : c->sb;
    const int n = term == 0 ? ni : nb;
    double* jv = c->jv + (long)term * 2 * c->jv_ld;
    if (n <= 0) continue;
    for (int l = 0; l < c->L; l++) {
      const LayerDesc& ld = c->nd.l[l];
      KP_TRY(jvp_layer(sp, s.zin_at(l), c->ldz[l], s.g_at(l), c->ldg[l], n, s.S, ld.h_in + 1,
                       ld.h_out, c->Delta + ld.off, wptr(c->delta, ld.off, c->esz_p),
                       c->jvp_part, jv, c->jv_ld, l > 0 ? 1 : 0, c->st));
    }
  }
  KP_TRY(kstar_finish(c->pp, c->jv, c->jv_ld, ni, c->jv + 2 * c->jv_ld, c->jv_ld, nb, c->Delta,
                      c->delta, c->grad, c->D, hp->lambda, c->loss, c->ctl, c->ctl + 1, theta,
                      info, c->st));
  return KP_OK;
}

// The step after the inversion.  part < 0: all of it; 0: the direction and the
// momentum only; 2: the choice of the step size and the update only (the line
// search's losses already in loss[2..], e.g. from a grouped batch launch).
static kp_status step_tail(kfac_pinn_ctx* c, void* theta, const void* xi, const void* yi,
                           int32_t ni, const void* xb, const void* yb, int32_t nb,
                           const kp_hparams* hp, kp_step_info* info, int part = -1) {
  const int ncand = hp->lr_mode == 1 ? hp->grid_max_exp - hp->grid_min_exp + 1 : 0;
  if (part <= 0) {
    // 4) Delta = -C g, momentum
    KP_TRY(kron_apply_batched(c->kdesc, c->L, c->k_mmax, c->k_nmax, c->st));
    if (hp->lr_mode == 2) return kstar_tail(c, theta, ni, nb, hp, info);
    KP_TRY(momentum(c->pp, c->Delta, c->delta, hp->momentum, c->ctl + 1, c->dhat, c->D, c->st));
    if (part == 0) return KP_OK;
  }
  if (part == 2) c->last_ncand = ncand;
  // 5) learning rate and update
  if (hp->lr_mode == 1 && part < 0) {
    // The candidates are independent: with two lanes the odd ones run on lane 1
    // (its own buffers, forked from and joined to the context's stream), so one
    // candidate's launches fill the chip while the other's drain.
    const bool two = c->ls_lanes == 2 && ncand > 1 && c->ls1.ready && c->eg_streams &&
                     c->eg.n > 1;
    if (two) {
      c->ls1.st = c->eg.st[1];
      KP_TRY(hipEventRecord(c->ls1.fork, c->st));
      KP_TRY(hipStreamWaitEvent(c->ls1.st, c->ls1.fork, 0));
    }
    for (int k = 0; k < ncand; k++) {
      const bool lane1 = two && (k & 1);
      if (lane1) ls_lane_swap(c);
      const double alpha = ldexp(1.0, hp->grid_max_exp - k);
      hipError_t e = axpy_theta(c->pp, theta, c->dhat, alpha, c->theta_trial, c->D, c->st);
      // the candidate's forward copy only: no backward copy, no BF16x3 low plane
      if (e == hipSuccess)
        e = prep_weights(c->lp == P_BF16 ? P_BF16 : c->wp, c->theta_trial, nullptr, 0.0, c->nd,
                         c->w_hi, nullptr, nullptr, 0, c->st, 1);
      if (e == hipSuccess) e = eval_loss(c, xi, yi, ni, xb, yb, nb, 2 + k);
      if (lane1) ls_lane_swap(c);
      KP_TRY(e);
    }
    if (two) {
      KP_TRY(hipEventRecord(c->ls1.join, c->ls1.st));
      KP_TRY(hipStreamWaitEvent(c->st, c->ls1.join, 0));
    }
    c->last_ncand = ncand;
  }
  KP_TRY(finish_step(c->pp, c->loss + 2, ncand, hp->grid_max_exp,
                     hp->lr_mode == 1 ? -1.0 : hp->lr, hp->momentum, c->loss, theta, c->dhat, c->delta, c->D,
                     c->ctl, c->ctl + 1, info, c->st));
  return KP_OK;
}

kp_status kfac_pinn_step(kfac_pinn_ctx* c, void* theta, const void* xi, const void* yi, int32_t ni,
                         const void* xb, const void* yb, int32_t nb, const kp_hparams* hp,
                         kp_step_info* info) {
  kp_status s = step_head(c, theta, xi, yi, ni, xb, yb, nb, hp);
  if (s != KP_OK) return s;
  // 3) preconditioner
  {
    int ti = tm_begin(c, KC_INVERT);
    KP_TRY(eig_all(c, hp->lambda));
    tm_end(c, ti, 0.0, 0.0);
  }
  return step_tail(c, theta, xi, yi, ni, xb, yb, nb, hp, info);
}

kp_status kfac_pinn_get_factor(kfac_pinn_ctx* c, int32_t layer, int32_t term, int32_t side,
                               double* out) {
  KP_ARG(c && out, "null argument");
  KP_ARG(layer >= 0 && layer < c->L && (term == 0 || term == 1) && (side == 0 || side == 1),
         "index out of range");
  const long n = side == 0 ? c->w[layer] + 1 : c->w[layer + 1];
  KP_TRY(hipMemcpyAsync(out, c->F[term][side][layer], sizeof(double) * n * n,
                        hipMemcpyDeviceToDevice, c->st));
  return KP_OK;
}

kp_status kfac_pinn_set_factor(kfac_pinn_ctx* c, int32_t layer, int32_t term, int32_t side,
                               const double* in) {
  KP_ARG(c && in, "null argument");
  KP_ARG(layer >= 0 && layer < c->L && (term == 0 || term == 1) && (side == 0 || side == 1),
         "index out of range");
  const long n = side == 0 ? c->w[layer] + 1 : c->w[layer + 1];
  KP_TRY(hipMemcpyAsync(c->F[term][side][layer], in, sizeof(double) * n * n,
                        hipMemcpyDeviceToDevice, c->st));
  return KP_OK;
}

kp_status kfac_pinn_get_preconditioner(kfac_pinn_ctx* c, int32_t layer, int32_t side, double* P,
                                       double* e) {
  KP_ARG(c, "null context");
  KP_ARG(layer >= 0 && layer < c->L && (side == 0 || side == 1), "index out of range");
  const EigProblem& p = c->probs[2 * layer + side];
  if (P)
    KP_TRY(hipMemcpyAsync(P, p.Pout, sizeof(double) * p.n * p.n, hipMemcpyDeviceToDevice, c->st));
  if (e) KP_TRY(hipMemcpyAsync(e, p.eout, sizeof(double) * p.n, hipMemcpyDeviceToDevice, c->st));
  return KP_OK;
}

kp_status kfac_pinn_get_line_search(kfac_pinn_ctx* c, double* out) {
  KP_ARG(c && out, "null argument");
  if (c->last_ncand > 0)
    KP_TRY(hipMemcpyAsync(out, c->loss + 2, sizeof(double) * c->last_ncand,
                          hipMemcpyDeviceToDevice, c->st));
  return KP_OK;
}

kp_status kfac_pinn_get_momentum(kfac_pinn_ctx* c, void* out) {
  KP_ARG(c && out, "null argument");
  KP_TRY(hipMemcpyAsync(out, c->delta, c->esz_p * c->D, hipMemcpyDeviceToDevice, c->st));
  return KP_OK;
}

kp_status kfac_pinn_set_momentum(kfac_pinn_ctx* c, const void* in, int64_t step) {
  KP_ARG(c && in, "null argument");
  KP_ARG(step >= 0 && step < (1LL << 30), "step out of range");
  KP_TRY(hipMemcpyAsync(c->delta, in, c->esz_p * c->D, hipMemcpyDeviceToDevice, c->st));
  static thread_local int stepv;
  stepv = (int)step;
  KP_TRY(hipMemcpyAsync(c->ctl + 1, &stepv, sizeof(int), hipMemcpyHostToDevice, c->st));
  KP_TRY(hipStreamSynchronize(c->st));
  return KP_OK;
}

kp_status kfac_pinn_timing_enable(kfac_pinn_ctx* c, int32_t kernel_class) {
  KP_ARG(c, "null context");
  KP_ARG(kernel_class >= -1 && kernel_class <= 4, "unknown kernel class");
  c->tm_cls = kernel_class;
  c->tm_used = 0;
  c->tm_flops = c->tm_bytes = 0.0;
  c->tm_launches = 0;
  return KP_OK;
}

kp_status kfac_pinn_timing_read(kfac_pinn_ctx* c, double* out) {
  KP_ARG(c && out, "null argument");
  KP_TRY(hipStreamSynchronize(c->st));
  double ms = 0.0;
  for (int i = 0; i + 1 < c->tm_used; i += 2) {
    float t = 0.f;
    KP_TRY(hipEventElapsedTime(&t, c->tm_ev[i], c->tm_ev[i + 1]));
    ms += t;
  }
  out[0] = (double)c->tm_launches;
  out[1] = ms;
  out[2] = c->tm_flops;
  out[3] = c->tm_bytes;
  c->tm_used = 0;
  c->tm_flops = c->tm_bytes = 0.0;
  c->tm_launches = 0;
  return KP_OK;
}

kp_status kfac_pinn_set_line_search_lanes(kfac_pinn_ctx* c, int32_t lanes) {
  KP_ARG(c, "null context");
  KP_ARG(lanes == 1 || lanes == 2, "lanes must be 1 or 2");
  KP_TRY(lanes == 2 ? ls_lane_alloc(c) : ls_lane_free(c));
  c->ls_lanes = lanes;
  return KP_OK;
}

kp_status kfac_pinn_get_sweeps(kfac_pinn_ctx* c, int32_t* out) {
  KP_ARG(c && out, "null argument");
  KP_TRY(hipStreamSynchronize(c->st));
  const int np = (int)c->probs.size();
  std::vector<int> flags(2 * np);
  KP_TRY(hipMemcpy(flags.data(), c->ctl + 8, sizeof(int) * 2 * np, hipMemcpyDeviceToHost));
  for (int q = 0; q < np; q++) out[q] = flags[2 * q + 1];
  return KP_OK;
}

kp_status kfac_pinn_get_workspace(kfac_pinn_ctx* c, int32_t* out) {
  KP_ARG(c && out, "null argument");
  out[0] = c->si.store ? 0 : 1;
  out[1] = c->sb.store ? 0 : 1;
  return KP_OK;
}

kp_status kfac_pinn_sync(kfac_pinn_ctx* c) {
  KP_ARG(c, "null context");
  KP_TRY(hipStreamSynchronize(c->st));
  int st = 0;
  KP_TRY(hipMemcpy(&st, c->ctl, sizeof(int), hipMemcpyDeviceToHost));
  if (st != 0) {
    int zero = 0;
    KP_TRY(hipMemcpy(c->ctl, &zero, sizeof(int), hipMemcpyHostToDevice));
  }
  return (kp_status)st;
}

// ---------------------------------------------------------------------------
// Batches of independent instances (one step of each per call).  Instance k
// runs on internal lane k % lanes, so the instances' small launches overlap.
// Each lane's part of the batch step is captured into its own HIP graph on the
// first call and replayed on later calls with the same arguments (different
// arguments recapture); one graph per lane keeps the lanes concurrent.
// ---------------------------------------------------------------------------
struct GroupChoice {
  int nch = 0;    // derivative-row chunks (0: the single-instance choice)
  int geo = -1;   // tile geometry (-1: the narrowest neuron tile covering the layer)
};

struct kfac_pinn_batch {
  std::vector<kfac_pinn_ctx*> ctx;
  hipStream_t st = nullptr;       // the caller's stream (may be the null stream)
  hipEvent_t ev_in = nullptr;     // fork: lanes wait for the caller's earlier work
  std::vector<hipStream_t> lanes;
  std::vector<hipEvent_t> ev_head;  // per lane: factors of its instances done
  hipEvent_t ev_eig = nullptr;      // the inversion of every instance done (lane 0)
  std::vector<hipEvent_t> ev;       // join: one per lane
  // graphs: per lane the heads and the tails of its instances, one inversion
  std::vector<hipGraph_t> graph;
  std::vector<hipGraphExec_t> exec_head, exec_tail;
  hipGraphExec_t exec_eig = nullptr;
  std::vector<uintptr_t> key;
  int use_graph = 1;
  // one inversion over the factors of every instance
  std::vector<EigProblem> probs;
  EigProblem* probs_dev = nullptr;
  EigGroups eg;             // one group: the inversion's launches already span every instance
  int* eig_ids = nullptr;
  int* eig_ctl = nullptr;   // [0..1] call counter and warm-start flag, [2..] 2 per problem
  // Grouped line search: each kernel of a candidate runs once over every instance
  // (job tables in device memory, sized at creation for the largest point counts
  // and rewritten when the step's buffers or point counts change).
  struct GTab {
    size_t jobs = 0, blk = 0;   // byte offsets in dev
    int njobs = 0, nblk = 0;
  };
  struct Group {
    GTab axpy, prep, slab, inq, inrows, loss;
    std::vector<std::array<GTab, kFwdGeos>> fwd;   // per hidden layer and tile geometry
    std::vector<GTab> fin;   // per hidden layer (fin[0] unused: the input layer's rows)
    char* dev = nullptr;
    size_t cap = 0;
    std::vector<uintptr_t> key;   // the step arguments the tables were built for
  } grp, grp1;   // grp1: the instances' second line-search buffers (odd candidates, lane 1)
  // Choices of the grouped layer products made by kfac_pinn_batch_tune, per class
  // (K, h_out, S, value rows only): the chunk count (0: the single-instance choice,
  // which gives the results of kfac_pinn_step) and the tile geometry (-1: by width).
  std::map<std::array<int, 4>, GroupChoice> tuned;
  // Grouped factor and gradient products: per (term, layer, product) one launch
  // of the split-K products over every instance and one of their reductions (in
  // the order of the single-instance backward sweep), on lane 0 before the
  // inversion; tables sized at creation, rewritten when point counts or beta change.
  struct PTab {
    GTab tn, red;
    int weighted = 0;
  };
  struct Prod {
    std::vector<PTab> pos;
    char* dev = nullptr;
    size_t cap = 0;
    int mode = 0;
    std::vector<uintptr_t> key;
  } prod;
  bool prod_active = false;
  int grouped = 1;          // use the grouped launches when every instance qualifies
  bool grp_active = false;  // this step's choice
  bool grp_two = false;     // with the odd candidates on lane 1
  std::vector<hipEvent_t> ev_pre;   // per lane: directions and momenta done
  hipEvent_t ev_ls = nullptr;       // grouped line search done (lane 0)
  hipEvent_t ev_ls1 = nullptr;      // its odd candidates done (lane 1)
  std::vector<hipGraphExec_t> exec_fin;
  hipGraphExec_t exec_ls = nullptr, exec_ls1 = nullptr;
};

namespace {
constexpr int kBatchLanes = 8;
constexpr int kMaxBatch = 1024;

void batch_drop_graph(kfac_pinn_batch* b) {
  for (hipGraphExec_t e : b->exec_head)
    if (e) (void)hipGraphExecDestroy(e);
  for (hipGraphExec_t e : b->exec_tail)
    if (e) (void)hipGraphExecDestroy(e);
  for (hipGraphExec_t e : b->exec_fin)
    if (e) (void)hipGraphExecDestroy(e);
  if (b->exec_eig) (void)hipGraphExecDestroy(b->exec_eig);
  if (b->exec_ls) (void)hipGraphExecDestroy(b->exec_ls);
  if (b->exec_ls1) (void)hipGraphExecDestroy(b->exec_ls1);
  for (hipGraph_t g : b->graph)
    if (g) (void)hipGraphDestroy(g);
  b->exec_head.clear();
  b->exec_tail.clear();
  b->exec_fin.clear();
  b->exec_eig = nullptr;
  b->exec_ls = nullptr;
  b->exec_ls1 = nullptr;
  b->graph.clear();
  b->key.clear();
}

struct BatchArgs {
  void* const* thetas;
  const void* const* xi;
  const void* const* yi;
  const int32_t* ni;
  const void* const* xb;
  const void* const* yb;
  const int32_t* nb;
  const kp_hparams* hp;
  kp_step_info* infos;
};

// Builds the grouped line search's job tables of every instance into `blob`
// (offsets into it in g).  bound: sizes only, for the largest point counts (the
// step's data pointers are not read).  False when an instance does not take the
// paired BF16 line search these kernels cover.
// Appends a job table and its workgroup list (largest jobs first: their tiles
// start in the first rounds, the small ones fill the tail) to blob.
void add_table(std::vector<char>& blob, kfac_pinn_batch::GTab& t, const void* jobs, size_t bytes,
               const std::vector<int>& nblk) {
  auto align = [&]() { blob.resize((blob.size() + 255) & ~(size_t)255); };
  align();
  t.jobs = blob.size();
  t.njobs = (int)nblk.size();
  blob.insert(blob.end(), (const char*)jobs, (const char*)jobs + bytes);
  std::vector<int> order(nblk.size());
  for (size_t j = 0; j < order.size(); j++) order[j] = (int)j;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nblk[x] > nblk[y]; });
  std::vector<GroupBlk> bl;
  for (int j : order)
    for (int i = 0; i < nblk[j]; i++) bl.push_back(GroupBlk{j, i});
  align();
  t.blk = blob.size();
  t.nblk = (int)bl.size();
  blob.insert(blob.end(), (const char*)bl.data(), (const char*)(bl.data() + bl.size()));
  align();
}

// The grouped factor and gradient products' tables (the arguments FactorGrad
// passes for every instance, term and layer).  bound: sizes for the largest point
// counts (every split count up to the cap).  False when an instance does not
// qualify (mixed curvature products, stored slabs, both point sets).
bool prod_build(kfac_pinn_batch* b, const int32_t* ni, const int32_t* nb, double beta, bool bound,
                std::vector<char>& blob, kfac_pinn_batch::Prod& pr) {
  const int n = (int)b->ctx.size();
  const int L = b->ctx[0]->L, mode = b->ctx[0]->cmode;
  if (mode != M_BF16X3 && mode != M_F16) return false;
  for (kfac_pinn_ctx* c : b->ctx)
    if (c->L != L || c->cmode != mode || !c->si.store || !c->sb.store) return false;
  pr.mode = mode;
  pr.pos.assign(2 * L * 3, kfac_pinn_batch::PTab{});
  blob.clear();
  std::vector<TnJob> tj(n);
  std::vector<RedJob> rj(n);
  std::vector<int> tnb(n), rnb(n);
  for (int t = 0; t < 2; t++)
    for (int l = L - 1; l >= 0; l--)
      for (int kind = 0; kind < 3; kind++) {
        for (int k = 0; k < n; k++) {
          kfac_pinn_ctx* c = b->ctx[k];
          const Slabs& s = t == 0 ? c->si : c->sb;
          const int np = bound ? (t == 0 ? c->max_i : c->max_b) : (t == 0 ? ni[k] : nb[k]);
          if (np <= 0) return false;
          const LayerDesc& ld = c->nd.l[l];
          const int K = np * s.S;
          const float* zin = (const float*)s.zin_at(l);
          const float* g = (const float*)s.g_at(l);
          const double sa = t == 0 ? 1.0 / ((double)np * s.S) : 1.0 / np, sbf = 1.0 / np;
          bool ok;
          if (kind == 0) {
            ok = make_tn_job(mode, zin, c->ldz[l], zin, c->ldz[l], ld.h_in + 1, ld.h_in + 1, K,
                             nullptr, np, true, (float*)c->part, kMaxSplits, c->wsc, &tj[k], &tnb[k]);
            rj[k] = make_red_job(tj[k], c->F[t][0][l], ld.h_in + 1, 1, (1.0 - beta) * sa, beta,
                                 &rnb[k]);
          } else if (kind == 1) {
            ok = make_tn_job(mode, g, c->ldg[l], g, c->ldg[l], ld.h_out, ld.h_out, K, nullptr, np,
                             true, (float*)c->part, kMaxSplits, c->wsc, &tj[k], &tnb[k]);
            rj[k] = make_red_job(tj[k], c->F[t][1][l], ld.h_out, 1, (1.0 - beta) * sbf, beta,
                                 &rnb[k]);
          } else {
            ok = make_tn_job(mode, g, c->ldg[l], zin, c->ldz[l], ld.h_out, ld.h_in + 1, K, s.rf, np,
                             false, (float*)c->part, kMaxSplits, c->wsc, &tj[k], &tnb[k]);
            rj[k] = make_red_job(tj[k], c->grad + ld.off, 1, ld.h_out, 1.0 / np,
                                 t == 0 ? 0.0 : 1.0, &rnb[k]);
          }
          if (!ok) return false;
          // sizes at creation: a smaller point count may take more splits
          if (bound) tnb[k] = 8 * (tj[k].sym ? tj[k].ntm * (tj[k].ntm + 1) / 2 : tj[k].ntm * tj[k].ntn) *
                              kp_cdiv(kMaxSplits, 8);
        }
        kfac_pinn_batch::PTab& p = pr.pos[(t * L + (L - 1 - l)) * 3 + kind];
        p.weighted = kind == 2;
        add_table(blob, p.tn, tj.data(), sizeof(TnJob) * n, tnb);
        add_table(blob, p.red, rj.data(), sizeof(RedJob) * n, rnb);
      }
  return true;
}

kp_status prod_run(kfac_pinn_batch* b, hipStream_t st) {
  const kfac_pinn_batch::Prod& pr = b->prod;
  char* d = pr.dev;
  for (const kfac_pinn_batch::PTab& p : pr.pos) {
    const TnJob* tj = (const TnJob*)(d + p.tn.jobs);
    if (p.weighted && pr.mode == M_F16) KP_TRY(row_scale_group(tj, p.tn.njobs, st));
    KP_TRY(tn_group(pr.mode, p.weighted != 0, tj, (const GroupBlk*)(d + p.tn.blk), p.tn.nblk, st));
    KP_TRY(reduce_group((const RedJob*)(d + p.red.jobs), (const GroupBlk*)(d + p.red.blk),
                        p.red.nblk, st));
  }
  return KP_OK;
}

typedef std::map<std::array<int, 4>, GroupChoice> ChoiceMap;
std::array<int, 4> group_class(const FwdLayerArgs& a) { return {a.K, a.h_out, a.S, a.value_only}; }

// the narrowest neuron tile that covers a layer of h_out neurons
int default_geo(int h_out) {
  int best = 0;
  for (int g = 0; g < kFwdGeos; g++)
    if (fwd_geo_width(g) >= h_out && fwd_geo_width(g) < fwd_geo_width(best)) best = g;
  return best;
}

bool group_build_set(kfac_pinn_batch* b, const BatchArgs* a, bool bound, std::vector<char>& blob,
                     kfac_pinn_batch::Group& g, const ChoiceMap* over);

// set 1: the tables over the instances' second line-search buffers
bool group_build(kfac_pinn_batch* b, const BatchArgs* a, bool bound, std::vector<char>& blob,
                 kfac_pinn_batch::Group& g, const ChoiceMap* over = nullptr, int set = 0) {
  if (set == 0) return group_build_set(b, a, bound, blob, g, over);
  for (kfac_pinn_ctx* c : b->ctx)
    if (!c->ls1.ready) return false;
  for (kfac_pinn_ctx* c : b->ctx) ls_lane_swap(c);
  const bool ok = group_build_set(b, a, bound, blob, g, over);
  for (kfac_pinn_ctx* c : b->ctx) ls_lane_swap(c);
  return ok;
}

bool group_build_set(kfac_pinn_batch* b, const BatchArgs* a, bool bound, std::vector<char>& blob,
                     kfac_pinn_batch::Group& g, const ChoiceMap* over) {
  if (!over) over = &b->tuned;
  const int n = (int)b->ctx.size();
  const int L = b->ctx[0]->L;
  if (L < 2) return false;
  std::vector<AxpyJob> ax(n);
  std::vector<PrepJob> pw(n);
  std::vector<SlabJob> sl(2 * n);
  std::vector<std::vector<FwdJob>> fw(L - 1, std::vector<FwdJob>(n));
  std::vector<std::vector<int>> fgeo(L - 1, std::vector<int>(n));
  std::vector<std::vector<FinJob>> fi(L - 1, std::vector<FinJob>(n));
  std::vector<InQJob> iq(n);
  std::vector<InRowsJob> ir(n);
  std::vector<LossJob> lo(n);
  std::vector<int> nax(n), npw(n), nsl(2 * n), niq(n), nir(n), nlo(n);
  std::vector<std::vector<int>> nfw(L - 1, std::vector<int>(n)), nfi(L - 1, std::vector<int>(n));
  auto blocks = [](long work, int cap) { return (int)std::max(1L, std::min<long>(cap, (work + 255) / 256)); };
  for (int k = 0; k < n; k++) {
    kfac_pinn_ctx* c = b->ctx[k];
    if (c->L != L || c->lp != P_BF16 || c->pp != P_F32 || c->nonlinear || c->dirs ||
        c->ls_lanes != 1 || !c->si.has_lap || c->sb.has_lap)
      return false;
    const int ni = bound ? c->max_i : a->ni[k], nb = bound ? c->max_b : a->nb[k];
    if (!ls_paired(c, ni, nb)) return false;
    FwdTarget Ti, Tb;
    ls_targets(c, Ti, Tb);
    ax[k] = AxpyJob{bound ? nullptr : (const float*)a->thetas[k], (const float*)c->dhat,
                    (float*)c->theta_trial, c->D, blocks(c->D, 128)};
    nax[k] = ax[k].nblk;
    long mx = 1;
    for (int l = 0; l < c->nd.L; l++)
      mx = std::max(mx, (long)c->nd.l[l].h_out * c->nd.l[l].ldk_in + c->nd.l[l].h_out);
    pw[k] = PrepJob{(const float*)c->theta_trial, c->w_hi, c->nd, blocks(mx, 64)};
    npw[k] = pw[k].nblk * c->nd.L;
    const int Si = input_rows_of(c, c->si, Ti), Sb = input_rows_of(c, c->sb, Tb);
    sl[2 * k] = SlabJob{bound ? nullptr : (const float*)a->xi[k], Ti.z(0), c->ldz[0], ni, c->d, Si,
                        blocks((long)ni * Si * c->ldz[0], 256)};
    sl[2 * k + 1] = SlabJob{bound ? nullptr : (const float*)a->xb[k], Tb.z(0), c->ldz[0], nb, c->d,
                            Sb, blocks((long)nb * Sb * c->ldz[0], 256)};
    nsl[2 * k] = sl[2 * k].nblk;
    nsl[2 * k + 1] = sl[2 * k + 1].nblk;
    for (int l = 0; l < L - 1; l++) {
      const LayerLaunch Li = layer_launch(c, c->si, ni, l, L, Ti);
      const LayerLaunch Lb = layer_launch(c, c->sb, nb, l, L, Tb);
      int nch = Li.nch, geo = default_geo(Li.a.h_out);
      auto it = over->find(group_class(Li.a));
      if (it != over->end()) {
        if (l > 0 && it->second.nch > 0) nch = it->second.nch;
        if (it->second.geo >= 0) geo = it->second.geo;
      }
      if (!make_fwd_job(Li.a, nch, Lb.a, geo, &fw[l][k])) return false;
      fgeo[l][k] = geo;
      // sizes at creation: the chunk count of a smaller step may be larger
      nfw[l][k] = bound ? fw[l][k].t0 * kMaxChunks + fw[l][k].t1 : fwd_job_blocks(fw[l][k]);
      if (l == 0) {
        if (!Li.input_rows || !make_input_jobs(Li.a, c->qbuf, 512, &iq[k], &ir[k])) return false;
        niq[k] = inq_job_blocks(iq[k]);
        nir[k] = ir[k].nblk;
      } else {
        if (Li.input_rows || !make_fin_job(Li.a, nch, &fi[l][k])) return false;
        nfi[l][k] = fin_job_blocks(fi[l][k]);
      }
    }
    const LayerDesc& ld = c->nd.l[L - 1];
    lo[k] = LossJob{Ti.z(L - 1), c->ldz[L - 1], ni, time_row_of(c, c->si), lap_row_of(c->si),
                    c->c_t, c->c_lap, bound ? nullptr : (const float*)a->yi[k], Tb.z(L - 1),
                    c->ldz[L - 1], nb, bound ? nullptr : (const float*)a->yb[k],
                    (const float*)wptr(c->theta_trial, ld.off, c->esz_p), ld.h_in + 1,
                    (ni + 3) / 4, ls_loss_blocks(ni, nb), c->partial, c->loss + 2};
    if (lo[k].nbt > c->partial_n) return false;
    nlo[k] = lo[k].nbt;
  }
  blob.clear();
  auto add = [&](kfac_pinn_batch::GTab& t, const void* jobs, size_t bytes,
                 const std::vector<int>& nblk) { add_table(blob, t, jobs, bytes, nblk); };
  add(g.axpy, ax.data(), sizeof(AxpyJob) * n, nax);
  add(g.prep, pw.data(), sizeof(PrepJob) * n, npw);
  add(g.slab, sl.data(), sizeof(SlabJob) * 2 * n, nsl);
  g.fwd.assign(L - 1, std::array<kfac_pinn_batch::GTab, kFwdGeos>{});
  g.fin.assign(L - 1, kfac_pinn_batch::GTab{});
  for (int l = 0; l < L - 1; l++) {
    // one table (one launch) per tile geometry in use
    for (int geo = 0; geo < kFwdGeos; geo++) {
      std::vector<FwdJob> jobs;
      std::vector<int> nbl;
      for (int k = 0; k < n; k++)
        if (fgeo[l][k] == geo) {
          jobs.push_back(fw[l][k]);
          nbl.push_back(nfw[l][k]);
        }
      add(g.fwd[l][geo], jobs.data(), sizeof(FwdJob) * jobs.size(), nbl);
    }
    if (l > 0) add(g.fin[l], fi[l].data(), sizeof(FinJob) * n, nfi[l]);
  }
  add(g.inq, iq.data(), sizeof(InQJob) * n, niq);
  add(g.inrows, ir.data(), sizeof(InRowsJob) * n, nir);
  add(g.loss, lo.data(), sizeof(LossJob) * n, nlo);
  return true;
}

// The grid line search of every instance, each kernel of a candidate one launch
// over all instances (the instances' own buffers, as their single-instance
// launches use them; the same kernels' bodies, so the losses are the same).
// parity < 0: every candidate on the tables of set 0; 0 / 1: the even / odd
// candidates on the tables of set 0 / 1.
kp_status group_ls(kfac_pinn_batch* b, const kp_hparams* hp, hipStream_t st, int parity = -1) {
  const kfac_pinn_batch::Group& g = parity == 1 ? b->grp1 : b->grp;
  char* d = g.dev;
  auto blk = [&](const kfac_pinn_batch::GTab& t) { return (const GroupBlk*)(d + t.blk); };
  const int ncand = hp->grid_max_exp - hp->grid_min_exp + 1;
  const int L = (int)g.fwd.size() + 1;
  for (int k = parity < 0 ? 0 : parity; k < ncand; k += parity < 0 ? 1 : 2) {
    const double alpha = ldexp(1.0, hp->grid_max_exp - k);
    KP_TRY(axpy_group((const AxpyJob*)(d + g.axpy.jobs), blk(g.axpy), g.axpy.nblk, alpha, st));
    KP_TRY(prep_group((const PrepJob*)(d + g.prep.jobs), blk(g.prep), g.prep.nblk, st));
    KP_TRY(slab_group((const SlabJob*)(d + g.slab.jobs), blk(g.slab), g.slab.nblk, st));
    for (int l = 0; l < L - 1; l++) {
      for (int geo = 0; geo < kFwdGeos; geo++)
        KP_TRY(fwd_group(geo, (const FwdJob*)(d + g.fwd[l][geo].jobs), blk(g.fwd[l][geo]),
                         g.fwd[l][geo].nblk, st));
      if (l == 0) {
        KP_TRY(inq_group((const InQJob*)(d + g.inq.jobs), blk(g.inq), g.inq.nblk, st));
        KP_TRY(inrows_group((const InRowsJob*)(d + g.inrows.jobs), blk(g.inrows), g.inrows.nblk,
                            st));
      } else {
        KP_TRY(fin_group((const FinJob*)(d + g.fin[l].jobs), blk(g.fin[l]), g.fin[l].nblk, st));
      }
    }
    KP_TRY(loss_group((const LossJob*)(d + g.loss.jobs), blk(g.loss), g.loss.nblk, st));
    KP_TRY(final_group((const LossJob*)(d + g.loss.jobs), g.loss.njobs, k, st));
  }
  return KP_OK;
}

// ---- autotuning of the grouped line search's layer products ------------------
// A cache entry: device, class (K, h_out, S, value rows only) and the choice
// (chunk count, 0: the single-instance choice; tile geometry).  The cache is a
// JSON file of these entries.
struct TuneEntry {
  std::string device;
  int K = 0, h_out = 0, S = 0, value_only = 0, nch = 0, geo = 0;
};

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t pr{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess)
    return "unknown";
  // the architecture and compute-unit count (the marketing name is not always
  // reported, e.g. under a profiler)
  std::string t = std::string(pr.gcnArchName) + " cu" + std::to_string(pr.multiProcessorCount);
  for (char& ch : t)
    if (ch == '"' || ch == '\\' || (unsigned char)ch < 32) ch = ' ';
  return t;
}

// Reads the flat objects of the cache's "entries" array (unknown keys skipped; a
// missing or malformed file, or an entry with a missing key, reads as absent).
std::vector<TuneEntry> tune_cache_read(const char* path) {
  std::vector<TuneEntry> out;
  if (!path) return out;
  FILE* f = fopen(path, "rb");
  if (!f) return out;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  fclose(f);
  size_t pos = txt.find("\"entries\"");
  while (pos != std::string::npos) {
    const size_t o = txt.find('{', pos), e = o == std::string::npos ? o : txt.find('}', o);
    if (o == std::string::npos || e == std::string::npos) break;
    const std::string obj = txt.substr(o + 1, e - o - 1);
    TuneEntry t;
    bool ok = true;
    auto num = [&](const char* key, int& v) {
      const size_t k = obj.find(std::string("\"") + key + "\"");
      const size_t c = k == std::string::npos ? k : obj.find(':', k);
      if (c == std::string::npos) ok = false;
      else v = atoi(obj.c_str() + c + 1);
    };
    num("K", t.K);
    num("h_out", t.h_out);
    num("S", t.S);
    num("value_only", t.value_only);
    num("nch", t.nch);
    num("geo", t.geo);
    const size_t k = obj.find("\"device\"");
    const size_t c = k == std::string::npos ? k : obj.find(':', k);
    const size_t q0 = c == std::string::npos ? c : obj.find('"', c);
    const size_t q1 = q0 == std::string::npos ? q0 : obj.find('"', q0 + 1);
    if (q1 == std::string::npos) ok = false;
    else t.device = obj.substr(q0 + 1, q1 - q0 - 1);
    if (ok && t.nch >= 0 && t.nch <= kMaxChunks && t.geo >= 0 && t.geo < kFwdGeos)
      out.push_back(t);
    pos = e + 1;
  }
  return out;
}

bool tune_cache_write(const char* path, const std::vector<TuneEntry>& es) {
  if (!path) return true;
  FILE* f = fopen(path, "wb");
  if (!f) return false;
  fprintf(f, "{\n  \"kfac_pinn_tune\": 2,\n  \"entries\": [\n");
  for (size_t i = 0; i < es.size(); i++)
    fprintf(f,
            "    {\"device\": \"%s\", \"K\": %d, \"h_out\": %d, \"S\": %d, "
            "\"value_only\": %d, \"nch\": %d, \"geo\": %d}%s\n",
            es[i].device.c_str(), es[i].K, es[i].h_out, es[i].S, es[i].value_only, es[i].nch,
            es[i].geo, i + 1 < es.size() ? "," : "");
  fprintf(f, "  ]\n}\n");
  return fclose(f) == 0;
}

// Chooses the tile geometry and chunk count of the grouped layer products by
// timing the grouped launches of every instance's layers (layer products, and
// the finishing passes past the input layer; minimum of 3 timed runs after one
// untimed).  First a policy for every class at once: the geometry by width or
// 64 x 256 everywhere, with the single-instance chunk counts or at most 1, 2, 4
// or 8 chunks (kept when at least 1 % faster in total).  Then class by class,
// within the launches of the layers the class occurs in, the other geometries
// and chunk counts (at most one per derivative row; kept when faster by more
// than 2 us and 0.5 %).  Classes in the cache for this device are taken from it.
kp_status batch_tune(kfac_pinn_batch* b, const BatchArgs& a, const char* cache_path,
                     int* timed_out) {
  hipStream_t st = b->lanes[0];
  ChoiceMap cur = b->tuned;
  std::vector<char> blob;
  kfac_pinn_batch::Group g = b->grp;
  if (!b->grp.dev || !group_build(b, &a, false, blob, g, &cur) || blob.size() > b->grp.cap)
    return KP_ERR_STATE;
  const int L = (int)g.fwd.size() + 1;
  // classes per layer, with their largest derivative-row count and their width
  struct ClassInfo {
    int nd = 0, h_out = 0;
  };
  std::vector<std::map<std::array<int, 4>, ClassInfo>> cls(L - 1);
  for (size_t k = 0; k < b->ctx.size(); k++) {
    kfac_pinn_ctx* c = b->ctx[k];
    FwdTarget Ti, Tb;
    ls_targets(c, Ti, Tb);
    for (int l = 0; l < L - 1; l++) {
      const LayerLaunch Li = layer_launch(c, c->si, a.ni[k], l, L, Ti);
      ClassInfo& ci = cls[l][group_class(Li.a)];
      ci.nd = std::max(ci.nd, Li.a.nd);
      ci.h_out = Li.a.h_out;
    }
  }
  const std::string dev = device_tag();
  std::vector<TuneEntry> cache = tune_cache_read(cache_path);
  auto cached = [&](const std::array<int, 4>& k) -> const TuneEntry* {
    for (const TuneEntry& t : cache)
      if (t.device == dev && t.K == k[0] && t.h_out == k[1] && t.S == k[2] && t.value_only == k[3])
        return &t;
    return nullptr;
  };
  // real slab contents for the timed launches: one line-search candidate (alpha = 1)
  KP_TRY(hipStreamSynchronize(st));
  KP_TRY(hipMemcpy(b->grp.dev, blob.data(), blob.size(), hipMemcpyHostToDevice));
  b->grp.key.clear();
  {
    kfac_pinn_batch::Group keep = b->grp;
    b->grp = g;
    b->grp.dev = keep.dev;
    b->grp.cap = keep.cap;
    kp_hparams one{};
    one.lr_mode = 1;
    one.grid_min_exp = 0;
    one.grid_max_exp = 0;
    kp_status s = group_ls(b, &one, st);
    b->grp = keep;
    if (s != KP_OK) return s;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  KP_TRY(hipEventCreate(&e0));
  KP_TRY(hipEventCreate(&e1));
  auto timed = [&](int l, float* ms) -> kp_status {
    kfac_pinn_batch::Group t = b->grp;
    if (!group_build(b, &a, false, blob, t, &cur) || blob.size() > b->grp.cap) return KP_ERR_STATE;
    KP_TRY(hipStreamSynchronize(st));
    KP_TRY(hipMemcpy(b->grp.dev, blob.data(), blob.size(), hipMemcpyHostToDevice));
    char* d = b->grp.dev;
    float best = 1e30f;
    for (int rep = 0; rep < 4; rep++) {
      KP_TRY(hipEventRecord(e0, st));
      for (int geo = 0; geo < kFwdGeos; geo++)
        KP_TRY(fwd_group(geo, (const FwdJob*)(d + t.fwd[l][geo].jobs),
                         (const GroupBlk*)(d + t.fwd[l][geo].blk), t.fwd[l][geo].nblk, st));
      if (l > 0)
        KP_TRY(fin_group((const FinJob*)(d + t.fin[l].jobs), (const GroupBlk*)(d + t.fin[l].blk),
                         t.fin[l].nblk, st));
      KP_TRY(hipEventRecord(e1, st));
      KP_TRY(hipEventSynchronize(e1));
      float v = 0.0f;
      KP_TRY(hipEventElapsedTime(&v, e0, e1));
      if (rep > 0) best = std::min(best, v);
    }
    *ms = best;
    return KP_OK;
  };
  // the classes to time (not in the cache), the layers each occurs in
  std::map<std::array<int, 4>, std::vector<int>> open_cls;
  std::map<std::array<int, 4>, ClassInfo> info;
  for (int l = 0; l < L - 1; l++)
    for (const auto& kv : cls[l]) {
      info[kv.first] = kv.second;
      if (const TuneEntry* t = cached(kv.first)) cur[kv.first] = GroupChoice{t->nch, t->geo};
      else open_cls[kv.first].push_back(l);
    }
  auto layers_ms = [&](const std::vector<int>& ls, float* ms) -> kp_status {
    float sum = 0.0f;
    for (int l : ls) {
      float v = 0.0f;
      kp_status s = timed(l, &v);
      if (s != KP_OK) return s;
      sum += v;
    }
    *ms = sum;
    return KP_OK;
  };
  std::vector<int> all_layers;
  for (int l = 0; l < L - 1; l++) all_layers.push_back(l);
  kp_status s = KP_OK;
  // 1) one policy for every open class
  auto policy = [&](bool by_width, int cap) {
    for (const auto& kv : open_cls) {
      const ClassInfo& ci = info[kv.first];
      const bool value_only = kv.first[3] != 0;
      cur[kv.first] = GroupChoice{value_only || cap == 0 ? 0 : std::min(cap, std::max(1, ci.nd)),
                                  by_width ? default_geo(ci.h_out) : 0};
    }
  };
  if (!open_cls.empty()) {
    bool best_w = true;
    int best_cap = 0;
    policy(true, 0);
    float best = 0.0f;
    s = layers_ms(all_layers, &best);
    for (int w = 1; w >= 0 && s == KP_OK; w--)
      for (int cap : {0, 1, 2, 4, 8}) {
        if (s != KP_OK || (w == 1 && cap == 0)) continue;
        policy(w == 1, cap);
        float v = 0.0f;
        if ((s = layers_ms(all_layers, &v)) == KP_OK && v < 0.99f * best) {
          best = v;
          best_w = w == 1;
          best_cap = cap;
        }
      }
    policy(best_w, best_cap);
  }
  // 2) class by class
  int ntimed = 0;
  for (const auto& kv : open_cls) {
    if (s != KP_OK) break;
    const std::array<int, 4>& key = kv.first;
    const ClassInfo& ci = info[key];
    GroupChoice ch = cur[key];
    float best = 0.0f;
    if ((s = layers_ms(kv.second, &best)) != KP_OK) break;
    std::vector<GroupChoice> alts;
    for (int geo = 0; geo < kFwdGeos; geo++)
      for (int nch : {0, 1, 2, 4, 8}) {
        if (key[3] != 0 && nch != 0) continue;   // the input layer's value rows: one chunk
        if (nch > std::max(1, ci.nd) || (geo == ch.geo && nch == ch.nch)) continue;
        alts.push_back(GroupChoice{nch, geo});
      }
    for (const GroupChoice& alt : alts) {
      cur[key] = alt;
      float v = 0.0f;
      if ((s = layers_ms(kv.second, &v)) != KP_OK) break;
      if (best - v > std::max(0.002f, 0.005f * best)) {
        best = v;
        ch = alt;
      }
    }
    if (s != KP_OK) break;
    cur[key] = ch;
    cache.push_back(TuneEntry{dev, key[0], key[1], key[2], key[3], ch.nch, ch.geo});
    ntimed++;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the step's tables are rebuilt (and its graphs recaptured) on the next call
  b->grp.key.clear();
  batch_drop_graph(b);
  if (s != KP_OK) return s;
  b->tuned = cur;
  if (timed_out) *timed_out = ntimed;
  if (!tune_cache_write(cache_path, cache)) {
    kp_set_last_error("cannot write the tuning cache", __FILE__, __LINE__);
    return KP_ERR_ARG;
  }
  return KP_OK;
}

// phase 0: the heads of the instances on lane l; 1: one inversion over every
// instance's problems on lane 0; 2: the tails of the instances on lane l (with the
// grouped line search: their directions and momenta); 3: the grouped line search
// of every instance on lane 0; 4: the step sizes and updates on lane l
kp_status batch_enqueue(kfac_pinn_batch* b, int phase, int l, const BatchArgs& a) {
  const int nl = (int)b->lanes.size();
  if (phase == 1) {
    if (b->prod_active) {
      kp_status s = prod_run(b, b->lanes[0]);
      if (s != KP_OK) return s;
    }
    int cap = 1;
    for (const kfac_pinn_ctx* c : b->ctx) cap = std::max(cap, c->max_sweeps);
    KP_TRY(kron_eig_batched(b->probs.data(), (int)b->probs.size(), a.hp->lambda, b->probs_dev,
                            b->ctx[0]->ctl, b->eig_ctl + 2, b->eig_ctl, kEigRefresh, cap, b->eg,
                            b->lanes[0]));
    return KP_OK;
  }
  // the grouped line search: all candidates on lane 0, or the even ones there and
  // the odd ones on lane 1 (phase 5), each lane's launch tails overlapping the other's
  if (phase == 3) return group_ls(b, a.hp, b->lanes[0], b->grp_two ? 0 : -1);
  if (phase == 5) return group_ls(b, a.hp, b->lanes[1], 1);
  const int part = phase == 2 ? (b->grp_active ? 0 : -1) : 2;
  for (size_t k = l; k < b->ctx.size(); k += nl) {
    kfac_pinn_ctx* c = b->ctx[k];
    kp_status s;
    if (phase == 0) {
      // with the grouped products the curvature passes leave them to phase 1
      c->defer_products = b->prod_active;
      s = step_head(c, a.thetas[k], a.xi[k], a.yi[k], a.ni[k], a.xb[k], a.yb[k], a.nb[k], a.hp);
      c->defer_products = false;
    } else {
      s = step_tail(c, a.thetas[k], a.xi[k], a.yi[k], a.ni[k], a.xb[k], a.yb[k], a.nb[k], a.hp,
                    a.infos ? a.infos + k : nullptr, part);
    }
    if (s != KP_OK) return s;
  }
  return KP_OK;
}

kp_status batch_capture(kfac_pinn_batch* b, int phase, int l, const BatchArgs& a,
                        hipGraphExec_t* out) {
  hipStream_t s = b->lanes[phase == 1 || phase == 3 ? 0 : phase == 5 ? 1 : l];
  KP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  kp_status st = batch_enqueue(b, phase, l, a);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (st != KP_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) kp_set_last_error(hipGetErrorString(e), __FILE__, __LINE__);
    return st != KP_OK ? st : KP_ERR_HIP;
  }
  b->graph.push_back(g);
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    *out = nullptr;
    kp_set_last_error(hipGetErrorString(e), __FILE__, __LINE__);
    return KP_ERR_HIP;
  }
  return KP_OK;
}

// The inversion's sweeps stop early when the host can read the convergence flags,
// which a captured graph cannot: then phase 1 is enqueued directly (each group's
// sweep still replays a graph of its own) and the other phases replay theirs.
bool batch_eig_direct(const kfac_pinn_batch* b) {
  return b->eg.host && b->eg.host_wait && b->eg.host_nprob == (int)b->probs.size();
}

kp_status batch_launch(kfac_pinn_batch* b, int phase, int l, const BatchArgs& a) {
  if (!b->use_graph || (phase == 1 && !b->exec_eig)) return batch_enqueue(b, phase, l, a);
  hipGraphExec_t x = phase == 0   ? b->exec_head[l]
                     : phase == 1 ? b->exec_eig
                     : phase == 2 ? b->exec_tail[l]
                     : phase == 3 ? b->exec_ls
                     : phase == 5 ? b->exec_ls1
                                  : b->exec_fin[l];
  KP_TRY(hipGraphLaunch(x, b->lanes[phase == 1 || phase == 3 ? 0 : phase == 5 ? 1 : l]));
  return KP_OK;
}
}  // namespace

kp_status kfac_pinn_batch_create(const kp_problem* problems, int32_t count, void* stream,
                                 kfac_pinn_batch** out) {
  KP_ARG(problems && out, "null argument");
  *out = nullptr;
  KP_ARG(count >= 1 && count <= kMaxBatch, "count must be in [1, 1024]");
  kfac_pinn_batch* b = new kfac_pinn_batch();
  b->st = (hipStream_t)stream;
  const int nl = count < kBatchLanes ? count : kBatchLanes;
  auto fail = [&](kp_status s) {
    kfac_pinn_batch_destroy(b);
    return s;
  };
  for (int l = 0; l < nl; l++) {
    hipStream_t s;
    hipEvent_t e, eh;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(KP_ERR_HIP);
    b->lanes.push_back(s);
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(KP_ERR_HIP);
    b->ev.push_back(e);
    if (hipEventCreateWithFlags(&eh, hipEventDisableTiming) != hipSuccess) return fail(KP_ERR_HIP);
    b->ev_head.push_back(eh);
    if (hipEventCreateWithFlags(&eh, hipEventDisableTiming) != hipSuccess) return fail(KP_ERR_HIP);
    b->ev_pre.push_back(eh);
  }
  if (hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_eig, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_ls, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_ls1, hipEventDisableTiming) != hipSuccess)
    return fail(KP_ERR_HIP);
  for (int k = 0; k < count; k++) {
    kfac_pinn_ctx* c = nullptr;
    kp_status s = kfac_pinn_create(&problems[k], b->lanes[k % nl], &c);
    if (s != KP_OK) return fail(s);
    // the batch's own lanes already overlap the instances: one line-search lane
    if ((s = kfac_pinn_set_line_search_lanes(c, 1)) != KP_OK) {
      kfac_pinn_destroy(c);
      return fail(s);
    }
    b->ctx.push_back(c);
    b->probs.insert(b->probs.end(), c->probs.begin(), c->probs.end());
  }
  const size_t np = b->probs.size();
  if (hipMalloc((void**)&b->probs_dev, sizeof(EigProblem) * np) != hipSuccess ||
      hipMalloc((void**)&b->eig_ids, sizeof(int) * np) != hipSuccess ||
      hipMalloc((void**)&b->eig_ctl, sizeof(int) * (2 + 2 * np)) != hipSuccess)
    return fail(KP_ERR_OOM);
  std::vector<int> ids(np);
  eig_groups_plan(b->probs.data(), (int)np, 1, ids.data(), b->eg);
  b->eg.ids = b->eig_ids;
  if (eig_host_sync(b->eg, ids.data(), (int)np) != hipSuccess) return fail(KP_ERR_HIP);
  if (hipMemcpy(b->probs_dev, b->probs.data(), sizeof(EigProblem) * np, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->eig_ids, ids.data(), sizeof(int) * np, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(b->eig_ctl, 0, sizeof(int) * (2 + 2 * np)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess)
    return fail(KP_ERR_HIP);
  {
    // the grouped line search's and products' tables, sized for the largest point counts
    std::vector<char> blob;
    if (group_build(b, nullptr, true, blob, b->grp)) {
      if (hipMalloc((void**)&b->grp.dev, blob.size()) != hipSuccess) return fail(KP_ERR_OOM);
      b->grp.cap = blob.size();
      // the second line-search buffers of every instance (odd candidates on lane
      // 1); without the memory for them the grouped line search keeps one lane
      bool ok = nl >= 2;
      for (kfac_pinn_ctx* c : b->ctx)
        if (ok && ls_lane_alloc(c) != hipSuccess) ok = false;
      if (!ok) {
        (void)hipGetLastError();
        for (kfac_pinn_ctx* c : b->ctx)
          if (ls_lane_free(c) != hipSuccess) return fail(KP_ERR_HIP);
      }
      if (ok && group_build(b, nullptr, true, blob, b->grp1, nullptr, 1)) {
        if (hipMalloc((void**)&b->grp1.dev, blob.size()) != hipSuccess) return fail(KP_ERR_OOM);
        b->grp1.cap = blob.size();
      }
    }
    if (prod_build(b, nullptr, nullptr, 0.0, true, blob, b->prod)) {
      if (hipMalloc((void**)&b->prod.dev, blob.size()) != hipSuccess) return fail(KP_ERR_OOM);
      b->prod.cap = blob.size();
    }
  }
  *out = b;
  return KP_OK;
}

kp_status kfac_pinn_batch_destroy(kfac_pinn_batch* b) {
  if (!b) return KP_ERR_ARG;
  for (hipStream_t s : b->lanes) (void)hipStreamSynchronize(s);
  batch_drop_graph(b);
  for (kfac_pinn_ctx* c : b->ctx) kfac_pinn_destroy(c);
  eig_host_free(b->eg);
  if (b->probs_dev) (void)hipFree(b->probs_dev);
  if (b->eig_ids) (void)hipFree(b->eig_ids);
  if (b->eig_ctl) (void)hipFree(b->eig_ctl);
  if (b->grp.dev) (void)hipFree(b->grp.dev);
  if (b->grp1.dev) (void)hipFree(b->grp1.dev);
  if (b->prod.dev) (void)hipFree(b->prod.dev);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->ev_head) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->ev_pre) (void)hipEventDestroy(e);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_eig) (void)hipEventDestroy(b->ev_eig);
  if (b->ev_ls) (void)hipEventDestroy(b->ev_ls);
  if (b->ev_ls1) (void)hipEventDestroy(b->ev_ls1);
  for (hipStream_t s : b->lanes) (void)hipStreamDestroy(s);
  delete b;
  return KP_OK;
}

kp_status kfac_pinn_batch_context(kfac_pinn_batch* b, int32_t k, kfac_pinn_ctx** out) {
  KP_ARG(b && out, "null argument");
  KP_ARG(k >= 0 && k < (int)b->ctx.size(), "instance index out of range");
  *out = b->ctx[k];
  return KP_OK;
}

kp_status kfac_pinn_batch_set_graph(kfac_pinn_batch* b, int32_t enabled) {
  KP_ARG(b, "null batch");
  b->use_graph = enabled ? 1 : 0;
  if (!enabled) batch_drop_graph(b);
  return KP_OK;
}

kp_status kfac_pinn_batch_set_grouped(kfac_pinn_batch* b, int32_t enabled) {
  KP_ARG(b, "null batch");
  KP_ARG(enabled == 0 || enabled == 1, "enabled must be 0 or 1");
  b->grouped = enabled;
  return KP_OK;
}

kp_status kfac_pinn_batch_tune(kfac_pinn_batch* b, void* const* thetas, const void* const* x_int,
                               const void* const* y_int, const int32_t* n_int,
                               const void* const* x_bnd, const void* const* y_bnd,
                               const int32_t* n_bnd, const char* cache_path, int32_t* timed) {
  KP_ARG(b && thetas && x_int && y_int && n_int && x_bnd && y_bnd && n_bnd, "null argument");
  const int n = (int)b->ctx.size();
  for (int k = 0; k < n; k++) {
    KP_ARG(n_int[k] > 0 && n_int[k] <= b->ctx[k]->max_i && n_bnd[k] > 0 &&
               n_bnd[k] <= b->ctx[k]->max_b,
           "point counts out of range (the grouped line search needs both point sets)");
    KP_ARG(thetas[k] && x_int[k] && y_int[k] && x_bnd[k] && y_bnd[k], "null buffer");
  }
  if (!b->grp.dev) {
    kp_set_last_error("the batch's instances do not take the grouped line search", __FILE__,
                      __LINE__);
    return KP_ERR_STATE;
  }
  // after the work already on the caller's stream
  KP_TRY(hipEventRecord(b->ev_in, b->st));
  KP_TRY(hipStreamWaitEvent(b->lanes[0], b->ev_in, 0));
  for (int l = 1; l < (int)b->lanes.size(); l++) KP_TRY(hipStreamSynchronize(b->lanes[l]));
  kp_hparams hp{};
  hp.lr_mode = 1;
  const BatchArgs a{thetas, x_int, y_int, n_int, x_bnd, y_bnd, n_bnd, &hp, nullptr};
  int t = 0;
  kp_status s = batch_tune(b, a, cache_path, &t);
  if (timed) *timed = t;
  KP_TRY(hipStreamSynchronize(b->lanes[0]));
  return s;
}

kp_status kfac_pinn_batch_is_grouped(kfac_pinn_batch* b, int32_t* out) {
  KP_ARG(b && out, "null argument");
  *out = (b->grp_active ? 1 : 0) | (b->prod_active ? 2 : 0) | (b->grp_two ? 4 : 0);
  return KP_OK;
}

kp_status kfac_pinn_batch_get_sweeps(kfac_pinn_batch* b, int32_t k, int32_t* sweeps) {
  KP_ARG(b && sweeps, "null argument");
  KP_ARG(k >= 0 && k < (int)b->ctx.size(), "instance index out of range");
  int first = 0;
  for (int i = 0; i < k; i++) first += (int)b->ctx[i]->probs.size();
  const int np = (int)b->ctx[k]->probs.size();
  std::vector<int> d(2 * np);
  KP_TRY(hipStreamSynchronize(b->lanes[0]));
  KP_TRY(hipMemcpy(d.data(), b->eig_ctl + 2 + 2 * first, sizeof(int) * 2 * np,
                   hipMemcpyDeviceToHost));
  for (int q = 0; q < np; q++) sweeps[q] = d[2 * q + 1];
  return KP_OK;
}

kp_status kfac_pinn_batch_step(kfac_pinn_batch* b, void* const* thetas, const void* const* x_int,
                               const void* const* y_int, const int32_t* n_int,
                               const void* const* x_bnd, const void* const* y_bnd,
                               const int32_t* n_bnd, const kp_hparams* hp, kp_step_info* infos) {
  KP_ARG(b && thetas && x_int && y_int && n_int && x_bnd && y_bnd && n_bnd && hp,
         "null argument");
  const int n = (int)b->ctx.size();
  const int nl = (int)b->lanes.size();
  const BatchArgs a{thetas, x_int, y_int, n_int, x_bnd, y_bnd, n_bnd, hp, infos};
  std::vector<uintptr_t> key;
  key.reserve(7 * n + 16);
  for (int k = 0; k < n; k++) {
    key.push_back((uintptr_t)thetas[k]);
    key.push_back((uintptr_t)x_int[k]);
    key.push_back((uintptr_t)y_int[k]);
    key.push_back((uintptr_t)x_bnd[k]);
    key.push_back((uintptr_t)y_bnd[k]);
    key.push_back((uintptr_t)n_int[k]);
    key.push_back((uintptr_t)n_bnd[k]);
  }
  // The grouped line search needs the grid search, tables for these arguments and
  // arguments every instance accepts (a failing instance reports from its head).
  b->grp_active = false;
  if (b->grouped && hp->lr_mode == 1 && b->grp.dev) {
    bool valid = true;
    for (int k = 0; k < n && valid; k++)
      valid = n_int[k] > 0 && n_int[k] <= b->ctx[k]->max_i && n_bnd[k] > 0 &&
              n_bnd[k] <= b->ctx[k]->max_b && x_int[k] && y_int[k] && x_bnd[k] && y_bnd[k] &&
              thetas[k];
    if (valid && key == b->grp.key) {
      b->grp_active = true;
    } else if (valid) {
      // nothing in flight may read the old tables (the grouped launches run on
      // lanes 0 and 1)
      KP_TRY(hipStreamSynchronize(b->lanes[0]));
      if (b->grp1.dev) KP_TRY(hipStreamSynchronize(b->lanes[1]));
      std::vector<char> blob;
      kfac_pinn_batch::Group g = b->grp;
      if (group_build(b, &a, false, blob, g) && blob.size() <= b->grp.cap) {
        KP_TRY(hipMemcpy(b->grp.dev, blob.data(), blob.size(), hipMemcpyHostToDevice));
        g.dev = b->grp.dev;
        g.cap = b->grp.cap;
        g.key = key;
        b->grp = g;
        b->grp_active = true;
        b->grp1.key.clear();
        kfac_pinn_batch::Group g1 = b->grp1;
        if (b->grp1.dev && group_build(b, &a, false, blob, g1, nullptr, 1) &&
            blob.size() <= b->grp1.cap) {
          KP_TRY(hipMemcpy(b->grp1.dev, blob.data(), blob.size(), hipMemcpyHostToDevice));
          g1.dev = b->grp1.dev;
          g1.cap = b->grp1.cap;
          g1.key = key;
          b->grp1 = g1;
        }
      }
    }
  }
  b->grp_two = b->grp_active && b->grp1.dev && b->grp1.key == b->grp.key &&
               hp->grid_max_exp > hp->grid_min_exp;
  // The grouped products need valid point counts and beta (their tables hold the
  // EMA weights); an invalid argument is reported by the instance's head.
  b->prod_active = false;
  if (b->grouped && b->prod.dev && hp->beta >= 0.0 && hp->beta < 1.0) {
    std::vector<uintptr_t> pkey;
    bool valid = true;
    for (int k = 0; k < n && valid; k++) {
      valid = n_int[k] > 0 && n_int[k] <= b->ctx[k]->max_i && n_bnd[k] > 0 &&
              n_bnd[k] <= b->ctx[k]->max_b;
      pkey.push_back((uintptr_t)n_int[k]);
      pkey.push_back((uintptr_t)n_bnd[k]);
    }
    uint64_t bb = 0;
    memcpy(&bb, &hp->beta, sizeof bb);
    pkey.push_back((uintptr_t)bb);
    if (valid && pkey == b->prod.key) {
      b->prod_active = true;
    } else if (valid) {
      std::vector<char> blob;
      kfac_pinn_batch::Prod pr = b->prod;
      if (prod_build(b, n_int, n_bnd, hp->beta, false, blob, pr) && blob.size() <= b->prod.cap) {
        KP_TRY(hipStreamSynchronize(b->lanes[0]));
        KP_TRY(hipMemcpy(b->prod.dev, blob.data(), blob.size(), hipMemcpyHostToDevice));
        pr.dev = b->prod.dev;
        pr.cap = b->prod.cap;
        pr.key = pkey;
        b->prod = pr;
        b->prod_active = true;
      }
    }
  }
  key.push_back((uintptr_t)infos);
  key.push_back((uintptr_t)b->grp_active);
  key.push_back((uintptr_t)b->grp_two);
  key.push_back((uintptr_t)b->prod_active);
  const bool eig_direct = batch_eig_direct(b);
  key.push_back((uintptr_t)eig_direct);
  {
    const unsigned char* hb = (const unsigned char*)hp;
    for (size_t i = 0; i < sizeof(kp_hparams); i++) key.push_back(hb[i]);
  }
  if (b->use_graph) {
    if (b->exec_head.empty() || key != b->key) {
      batch_drop_graph(b);
      b->exec_head.assign(nl, nullptr);
      b->exec_tail.assign(nl, nullptr);
      b->exec_fin.assign(nl, nullptr);
      kp_status s = KP_OK;
      for (int l = 0; l < nl && s == KP_OK; l++) s = batch_capture(b, 0, l, a, &b->exec_head[l]);
      if (s == KP_OK && !eig_direct) s = batch_capture(b, 1, 0, a, &b->exec_eig);
      for (int l = 0; l < nl && s == KP_OK; l++) s = batch_capture(b, 2, l, a, &b->exec_tail[l]);
      if (b->grp_active) {
        if (s == KP_OK) s = batch_capture(b, 3, 0, a, &b->exec_ls);
        if (s == KP_OK && b->grp_two) s = batch_capture(b, 5, 1, a, &b->exec_ls1);
        for (int l = 0; l < nl && s == KP_OK; l++) s = batch_capture(b, 4, l, a, &b->exec_fin[l]);
      }
      if (s != KP_OK) {
        batch_drop_graph(b);
        return s;
      }
      b->key = key;
    }
  }
  // ordered after the caller's earlier work and before its later work: heads on
  // every lane, the inversion on lane 0 after all heads, tails after it
  KP_TRY(hipEventRecord(b->ev_in, b->st));
  for (int l = 0; l < nl; l++) {
    KP_TRY(hipStreamWaitEvent(b->lanes[l], b->ev_in, 0));
    kp_status s = batch_launch(b, 0, l, a);
    if (s != KP_OK) return s;
    KP_TRY(hipEventRecord(b->ev_head[l], b->lanes[l]));
  }
  for (int l = 1; l < nl; l++) KP_TRY(hipStreamWaitEvent(b->lanes[0], b->ev_head[l], 0));
  {
    kp_status s = batch_launch(b, 1, 0, a);
    if (s != KP_OK) return s;
  }
  KP_TRY(hipEventRecord(b->ev_eig, b->lanes[0]));
  for (int l = 0; l < nl; l++) {
    if (l > 0) KP_TRY(hipStreamWaitEvent(b->lanes[l], b->ev_eig, 0));
    kp_status s = batch_launch(b, 2, l, a);
    if (s != KP_OK) return s;
    if (b->grp_active) {
      KP_TRY(hipEventRecord(b->ev_pre[l], b->lanes[l]));
      continue;
    }
    KP_TRY(hipEventRecord(b->ev[l], b->lanes[l]));
    KP_TRY(hipStreamWaitEvent(b->st, b->ev[l], 0));
  }
  if (!b->grp_active) return KP_OK;
  // the grouped line search on lane 0 after every lane's directions, then the
  // step sizes and updates back on the lanes
  for (int l = 1; l < nl; l++) KP_TRY(hipStreamWaitEvent(b->lanes[0], b->ev_pre[l], 0));
  if (b->grp_two)
    for (int l = 0; l < nl; l++)
      if (l != 1) KP_TRY(hipStreamWaitEvent(b->lanes[1], b->ev_pre[l], 0));
  {
    kp_status s = batch_launch(b, 3, 0, a);
    if (s != KP_OK) return s;
    if (b->grp_two && (s = batch_launch(b, 5, 1, a)) != KP_OK) return s;
  }
  KP_TRY(hipEventRecord(b->ev_ls, b->lanes[0]));
  if (b->grp_two) KP_TRY(hipEventRecord(b->ev_ls1, b->lanes[1]));
  for (int l = 0; l < nl; l++) {
    if (l > 0) KP_TRY(hipStreamWaitEvent(b->lanes[l], b->ev_ls, 0));
    if (b->grp_two && l != 1) KP_TRY(hipStreamWaitEvent(b->lanes[l], b->ev_ls1, 0));
    kp_status s = batch_launch(b, 4, l, a);
    if (s != KP_OK) return s;
    KP_TRY(hipEventRecord(b->ev[l], b->lanes[l]));
    KP_TRY(hipStreamWaitEvent(b->st, b->ev[l], 0));
  }
  return KP_OK;
}

}  // extern "C"
