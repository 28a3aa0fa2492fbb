// FP64 linear algebra for the inverse of the damped Kronecker sum (Section 3.4).
//
// For every layer and side the pair (F1, F2) = (damped interior factor, damped
// boundary factor) is brought to P^T F1 P = I, P^T F2 P = diag(e):
//   1. blocked Cholesky F1 = L L^T (64 x 64 blocks),
//   2. blocked triangular inverse L^-1,
//   3. M = L^-1 F2 L^-T (two products),
//   4. two-sided block Jacobi on C = V0^T M V0 (32-wide blocks, round-robin
//      pairing of block pairs; each pair's 64 x 64 subproblem gets one sweep
//      of parallel Jacobi rotations in LDS (all index pairs in the first round
//      of an outer sweep, the pairs across the two blocks in the others), then
//      the rotations are applied to C and accumulated into V), until a sweep
//      performs no rotation above the threshold.  The problems are split into
//      groups whose rounds run on separate streams.  V0 is the identity on a cold start; on a warm start it is
//      the previous call's V, the eigenvectors of the previous whitened
//      matrix: the factors move slowly under the moving average, so C starts
//      nearly diagonal and few sweeps remain,
//   5. e = diag(C), P = L^-T V.
// The inverse of A1 (x) B1 + A2 (x) B2 is then (P_A (x) P_B)(I + e_A (x) e_B)^-1
// (P_A (x) P_B)^T.  Every problem is padded to a multiple of 64 with an identity
// block in F1 and a zero block in F2, which stays exactly decoupled (V keeps
// the block structure).  All problems of a call run in the same launches
// (grid.y = problem).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.h"
#include "launch.h"

namespace kp {

constexpr int BB = 64;        // Cholesky / inverse block
constexpr int LDB = BB + 1;   // LDS row stride (doubles)
constexpr int JB = 32;        // Jacobi block

// 64 x 64 x 64 FP64 products on the MFMA unit (v_mfma_f64_16x16x4): four waves,
// each owning a 32 x 32 quadrant as 2 x 2 tiles of 16 x 16.  Tiles sit in LDS
// with row stride LDM = 70 doubles, which keeps the fragment reads at two
// (16 rows x 4 k) or three (4 k x 16 columns) accesses per bank.
constexpr int LDM = 70;

// acc[ti][tj] += op(A) op(B) over k in [0, 64); op(A)[i][k] = TA ? A[k][i] : A[i][k],
// op(B)[k][j] = TB ? B[j][k] : B[k][j].  Element (r) of acc[ti][tj] is output
// (32 wi + 16 ti + (lane >> 4) + 4 r, 32 wj + 16 tj + (lane & 15)).
template <bool TA, bool TB>
__device__ __forceinline__ void mm64(f64x4 (&acc)[2][2], const double* A, const double* B) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1, r16 = lane & 15, kq = lane >> 4;
#pragma unroll 4
  for (int k0 = 0; k0 < 64; k0 += 4) {
    const int k = k0 + kq;
    double a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; t++) {
      const int i = 32 * wi + 16 * t + r16, j = 32 * wj + 16 * t + r16;
      a[t] = TA ? A[k * LDM + i] : A[i * LDM + k];
      b[t] = TB ? B[j * LDM + k] : B[k * LDM + j];
    }
#pragma unroll
    for (int ti = 0; ti < 2; ti++)
#pragma unroll
      for (int tj = 0; tj < 2; tj++) acc[ti][tj] = Mfma<double>::mma(a[ti], b[tj], acc[ti][tj]);
  }
}

__device__ __forceinline__ void mm64_zero(f64x4 (&acc)[2][2]) {
#pragma unroll
  for (int ti = 0; ti < 2; ti++)
#pragma unroll
    for (int tj = 0; tj < 2; tj++) acc[ti][tj] = f64x4{0.0, 0.0, 0.0, 0.0};
}

// Visit the outputs of this thread: f(i, j, value) in tile coordinates.
template <class F>
__device__ __forceinline__ void mm64_each(const f64x4 (&acc)[2][2], F f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
#pragma unroll
  for (int ti = 0; ti < 2; ti++)
#pragma unroll
    for (int tj = 0; tj < 2; tj++)
#pragma unroll
      for (int r = 0; r < 4; r++)
        f(32 * wi + 16 * ti + Mfma<double>::row(lane, r), 32 * wj + 16 * tj + (lane & 15),
          acc[ti][tj][r]);
}

// ---------------------------------------------------------------------------
// 0. damping and padding
// ---------------------------------------------------------------------------
__global__ void k_damp_pad(const EigProblem* __restrict__ pr, double lambda) {
  const EigProblem p = pr[blockIdx.y];
  const long np2 = (long)p.n_pad * p.n_pad;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < np2;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / p.n_pad), j = (int)(e % p.n_pad);
    double a = 0.0, b = 0.0;
    if (i < p.n && j < p.n) {
      a = p.f1[(long)i * p.n + j];
      b = p.f2[(long)i * p.n + j];
      if (i == j) { a += lambda; b += lambda; }
    } else if (i == j) {
      a = 1.0;
    }
    p.M1[e] = a;
    p.M2[e] = b;
    p.Lb[e] = 0.0;
    p.Li[e] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// 1. Cholesky: diagonal block (factor + inverse of the factor)
//
// Right-looking elimination with the inverse carried along: thread (ty, tx)
// keeps the 16 elements (ty + 16 a, tx + 16 b) of the tile in registers.  At
// step k the pivot column k of the Schur complement W and row k of R (the
// rows of the identity reduced by the finished columns, L X = I solved
// forward) are published in LDS; then
//   L[i][k] = W[i][k] / d_k (d_k = sqrt W[k][k]),  X[k][c] = R[k][c] / d_k,
//   W[i][c] -= W[i][k] W[c][k] / W[k][k]           (k < c <= i),
//   R[i][c] -= W[i][k] R[k][c] / W[k][k]           (c <= k < i),
// and an element leaves W for R when its column is finished.  The column and
// row of step k + 1 are published into the other LDS buffer, so a step takes
// one barrier; the results stay in registers until the end (a global store
// before a barrier would make every step wait for it).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chol_diag(const EigProblem* __restrict__ pr, int j,
                                                   int* status) {
  const EigProblem p = pr[blockIdx.y];
  const int nb = p.n_pad / BB;
  if (j >= nb) return;
  __shared__ double colk[2][BB];
  __shared__ double rowk[2][BB];
  __shared__ double LO[BB * LDB];   // L, filled a column per step
  __shared__ double XO[BB * LDB];   // L^-1, filled a row per step
  const long np = p.n_pad;
  const double* src = p.M1 + (long)j * BB * np + (long)j * BB;
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  // Elements above the diagonal are loaded as zero and later take values that
  // nothing reads: the published entries above row k + 1 of the column and
  // right of column k + 1 of the row are never used.
  double v[4][4];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) {
      const int i = ty + 16 * a, c = tx + 16 * b;
      v[a][b] = c <= i ? src[(long)i * np + c] : 0.0;
      if (c == 0) colk[0][i] = v[a][b];
      if (i == 0) rowk[0][c] = c == 0 ? 1.0 : 0.0;
    }
  bool bad = false;
  for (int k = 0; k < BB; k++) {
    const int par = k & 1;
    __syncthreads();
    double piv = colk[par][k];
    if (!(piv > 0.0)) { bad = true; piv = 1.0; }
    const double dk = sqrt(piv), idk = 1.0 / dk, ip = idk * idk;
    if (threadIdx.x < BB) {   // column k of L
      const int i = threadIdx.x;
      LO[i * LDB + k] = i < k ? 0.0 : (i == k ? dk : colk[par][i] * idk);
    } else if (threadIdx.x < 2 * BB) {   // row k of L^-1 (R[k][k] = 1)
      const int c = threadIdx.x - BB;
      XO[k * LDB + c] = c > k ? 0.0 : rowk[par][c] * idk;
    }
    double oc[4];
#pragma unroll
    for (int b = 0; b < 4; b++) {
      const int c = tx + 16 * b;
      oc[b] = c > k ? colk[par][c] : rowk[par][c];
    }
#pragma unroll
    for (int a = 0; a < 4; a++) {
      const int i = ty + 16 * a;
      const double f = i > k ? colk[par][i] * ip : 0.0;
      const double eik = i == k ? 1.0 : 0.0;
#pragma unroll
      for (int b = 0; b < 4; b++) {
        const double x = tx + 16 * b == k ? eik : v[a][b];
        v[a][b] = x - f * oc[b];
      }
    }
    // publish the pivot column and R row of step k + 1 (static register
    // indices: a dynamic one would put v in scratch memory)
    const int k1 = k + 1;
#pragma unroll
    for (int b = 0; b < 4; b++)
      if (tx + 16 * b == k1)
#pragma unroll
        for (int a = 0; a < 4; a++) colk[par ^ 1][ty + 16 * a] = v[a][b];
#pragma unroll
    for (int a = 0; a < 4; a++)
      if (ty + 16 * a == k1)
#pragma unroll
        for (int b = 0; b < 4; b++) rowk[par ^ 1][tx + 16 * b] = tx + 16 * b == k1 ? 1.0 : v[a][b];
  }
  __syncthreads();
  double* lb = p.Lb + (long)j * BB * np + (long)j * BB;
  double* li = p.Li + (long)j * BB * np + (long)j * BB;
  for (int e = threadIdx.x; e < BB * BB; e += blockDim.x) {
    const int i = e / BB, c = e % BB;
    lb[(long)i * np + c] = LO[i * LDB + c];
    li[(long)i * np + c] = XO[i * LDB + c];
  }
  if (threadIdx.x == 0 && bad) atomicMax(p.status ? p.status : status, 4);
}

// Panel and trailing update of step j: workgroup (i, k), j <= k <= i, i > j.
//   L_ij = A_ij (L_jj^-1)^T;  for k > j: A_ik -= L_ij L_kj^T.
__global__ __launch_bounds__(256) void k_chol_update(const EigProblem* __restrict__ pr, int j) {
  const EigProblem p = pr[blockIdx.y];
  const int nb = p.n_pad / BB;
  if (j >= nb - 1) return;
  int w = blockIdx.x, i = j + 1, k;
  {
    int rowlen = 2;   // row i has (i - j + 1) blocks k = j..i
    while (w >= rowlen) { w -= rowlen; i++; rowlen++; }
    if (i >= nb) return;
    k = j + w;
  }
  __shared__ __align__(16) double T[BB * LDM];   // L_jj^-1
  __shared__ __align__(16) double Ai[BB * LDM];
  __shared__ __align__(16) double Ak[BB * LDM];
  const long np = p.n_pad;
  auto load = [&](double* dst, const double* src) {
    for (int e = threadIdx.x; e < BB * BB / 2; e += blockDim.x) {
      const int r = e >> 5, c = 2 * (e & 31);
      *(double2*)&dst[r * LDM + c] = *(const double2*)(src + (long)r * np + c);
    }
  };
  const bool two = k > j && k != i;
  load(T, p.Li + (long)j * BB * np + (long)j * BB);
  load(Ai, p.M1 + (long)i * BB * np + (long)j * BB);
  if (two) load(Ak, p.M1 + (long)k * BB * np + (long)j * BB);
  __syncthreads();
  f64x4 li[2][2], lk[2][2];
  mm64_zero(li);
  mm64<false, true>(li, Ai, T);
  if (two) {
    mm64_zero(lk);
    mm64<false, true>(lk, Ak, T);
  }
  __syncthreads();
  mm64_each(li, [&](int a, int b, double v) { Ai[a * LDM + b] = v; });
  if (two) mm64_each(lk, [&](int a, int b, double v) { Ak[a * LDM + b] = v; });
  __syncthreads();
  if (k == j) {
    double* dst = p.Lb + (long)i * BB * np + (long)j * BB;
    for (int e = threadIdx.x; e < BB * BB; e += blockDim.x)
      dst[(long)(e / BB) * np + (e % BB)] = Ai[(e / BB) * LDM + (e % BB)];
    return;
  }
  f64x4 acc[2][2];
  mm64_zero(acc);
  mm64<false, true>(acc, Ai, (k == i) ? Ai : Ak);
  double* dst = p.M1 + (long)i * BB * np + (long)k * BB;
  mm64_each(acc, [&](int a, int b, double v) { dst[(long)a * np + b] -= v; });
}

// ---------------------------------------------------------------------------
// 2. Triangular inverse, block row i:  Li_ij = -Li_ii sum_{k=j}^{i-1} L_ik Li_kj
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_trtri_row(const EigProblem* __restrict__ pr, int i) {
  const EigProblem p = pr[blockIdx.y];
  const int nb = p.n_pad / BB;
  const int j = blockIdx.x;
  if (i >= nb || j >= i) return;
  __shared__ __align__(16) double A[BB * LDM];
  __shared__ __align__(16) double B[BB * LDM];
  const long np = p.n_pad;
  auto load = [&](double* dst, const double* src) {
    for (int e = threadIdx.x; e < BB * BB / 2; e += blockDim.x) {
      const int r = e >> 5, c = 2 * (e & 31);
      *(double2*)&dst[r * LDM + c] = *(const double2*)(src + (long)r * np + c);
    }
  };
  f64x4 acc[2][2];
  mm64_zero(acc);
  for (int k = j; k < i; k++) {
    __syncthreads();
    load(A, p.Lb + (long)i * BB * np + (long)k * BB);
    load(B, p.Li + (long)k * BB * np + (long)j * BB);
    __syncthreads();
    mm64<false, false>(acc, A, B);
  }
  __syncthreads();
  mm64_each(acc, [&](int a, int b, double v) { B[a * LDM + b] = v; });
  load(A, p.Li + (long)i * BB * np + (long)i * BB);
  __syncthreads();
  mm64_zero(acc);
  mm64<false, false>(acc, A, B);
  double* dst = p.Li + (long)i * BB * np + (long)j * BB;
  mm64_each(acc, [&](int a, int b, double v) { dst[(long)a * np + b] = -v; });
}

// ---------------------------------------------------------------------------
// Batched FP64 products over 64 x 64 tiles (n_pad x n_pad operands):
//   mode 0: C1 <- Li F2          (F2 symmetric; Li lower: k <= bi)
//   mode 1: C0 <- C1 Li^T        (k <= bj)
//   mode 2: C1 <- C0 V           (warm start, V = P0)
//   mode 3: C0 <- V^T C1
//   mode 4: P1 <- Li^T V         (Li^T upper: k >= bi)
// ---------------------------------------------------------------------------
// The operand tiles of block k for output tile (bi, bj), by mode (a template
// parameter, so that the pointers need no run-time dispatch).
template <int MODE>
__device__ __forceinline__ const double* eig_mm_a(const EigProblem& p, long np, int bi, int k) {
  if constexpr (MODE == 0) return p.Li + (long)bi * BB * np + (long)k * BB;
  if constexpr (MODE == 1) return p.C[1] + (long)bi * BB * np + (long)k * BB;
  if constexpr (MODE == 2) return p.C[0] + (long)bi * BB * np + (long)k * BB;
  if constexpr (MODE == 3) return p.P[0] + (long)k * BB * np + (long)bi * BB;
  return p.Li + (long)k * BB * np + (long)bi * BB;
}
template <int MODE>
__device__ __forceinline__ const double* eig_mm_b(const EigProblem& p, long np, int bj, int k) {
  if constexpr (MODE == 0) return p.M2 + (long)bj * BB * np + (long)k * BB;
  if constexpr (MODE == 1) return p.Li + (long)bj * BB * np + (long)k * BB;
  if constexpr (MODE == 2) return p.P[0] + (long)k * BB * np + (long)bj * BB;
  if constexpr (MODE == 3) return p.C[1] + (long)k * BB * np + (long)bj * BB;
  return p.P[0] + (long)k * BB * np + (long)bj * BB;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_eig_mm(const EigProblem* __restrict__ pr,
                                                const int* __restrict__ warm) {
  if (MODE >= 2 && MODE <= 3 && !*warm) return;   // the warm-start products only
  const EigProblem p = pr[blockIdx.z];
  const int nb = p.n_pad / BB;
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi >= nb || bj >= nb) return;
  const long np = p.n_pad;
  __shared__ __align__(16) double As[BB * LDM];
  __shared__ __align__(16) double Bs[BB * LDM];
  // thread t moves elements 2t + 512 m (m < 8) of a tile: rows 8m + t / 32,
  // columns 2 (t % 32) and the next
  const int lr = threadIdx.x >> 5, lc = 2 * (threadIdx.x & 31);
  // native 2-vectors (HIP's double2 struct arrays are not kept in registers)
  typedef double d2 __attribute__((ext_vector_type(2)));
  d2 ra[8], rb[8];
  f64x4 acc[2][2];
  mm64_zero(acc);
  const int kbeg = MODE == 4 ? bi : 0;
  const int kend = MODE == 0 ? bi : (MODE == 1 ? bj : nb - 1);
  {
    const double* a = eig_mm_a<MODE>(p, np, bi, kbeg);
    const double* b = eig_mm_b<MODE>(p, np, bj, kbeg);
#pragma unroll
    for (int m = 0; m < 8; m++) {
      ra[m] = *(const d2*)(a + (long)(8 * m + lr) * np + lc);
      rb[m] = *(const d2*)(b + (long)(8 * m + lr) * np + lc);
    }
  }
  for (int k = kbeg; k <= kend; k++) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; m++) {
      *(d2*)&As[(8 * m + lr) * LDM + lc] = ra[m];
      *(d2*)&Bs[(8 * m + lr) * LDM + lc] = rb[m];
    }
    __syncthreads();
    if (k < kend) {   // the next tiles are in flight during the products
      const double* a = eig_mm_a<MODE>(p, np, bi, k + 1);
      const double* b = eig_mm_b<MODE>(p, np, bj, k + 1);
#pragma unroll
      for (int m = 0; m < 8; m++) {
        ra[m] = *(const d2*)(a + (long)(8 * m + lr) * np + lc);
        rb[m] = *(const d2*)(b + (long)(8 * m + lr) * np + lc);
      }
    }
    if constexpr (MODE <= 1) mm64<false, true>(acc, As, Bs);
    else if constexpr (MODE == 2) mm64<false, false>(acc, As, Bs);
    else mm64<true, false>(acc, As, Bs);   // modes 3 and 4: the A tile transposed
  }
  double* out = (MODE == 0 || MODE == 2) ? p.C[1] : (MODE == 4 ? p.P[1] : p.C[0]);
  out += (long)bi * BB * np + (long)bj * BB;
  mm64_each(acc, [&](int i, int j, double v) { out[(long)i * np + j] = v; });
}

// Call counter and warm-start flag, decided on the device so that a captured
// graph keeps the refresh schedule: calls[0] counts calls, calls[1] = warm.
__global__ void k_eig_begin(int* calls, int refresh) {
  const int n = calls[0];
  calls[1] = (n % refresh) != 0;
  calls[0] = n + 1;
}

// C <- (C + C^T)/2, V <- I on a cold start (kept on a warm start), flags reset
__global__ void k_jac_init(const EigProblem* __restrict__ pr, int* done, const int* warmp) {
  const int warm = *warmp;
  const EigProblem p = pr[blockIdx.y];
  const long np = p.n_pad;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < np * np;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / np), j = (int)(e % np);
    if (!warm) p.P[0][e] = i == j ? 1.0 : 0.0;
    if (j > i) {
      const double v = 0.5 * (p.C[0][e] + p.C[0][(long)j * np + i]);
      p.C[0][e] = v;
      p.C[0][(long)j * np + i] = v;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    done[2 * blockIdx.y] = 0;
    done[2 * blockIdx.y + 1] = 0;
    p.pflag[p.n_pad / 64] = 0;   // rotation flag of the sweep
  }
}

__global__ void k_jac_dmax(const EigProblem* __restrict__ pr) {
  const EigProblem p = pr[blockIdx.x];
  double m = 0.0;
  for (int i = threadIdx.x; i < p.n_pad; i += blockDim.x)
    m = fmax(m, fabs(p.C[0][(long)i * p.n_pad + i]));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  __shared__ double r[4];
  if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) *p.dmax = fmax(fmax(r[0], r[1]), fmax(r[2], r[3]));
}

// ---------------------------------------------------------------------------
// 4. Block Jacobi (in place).  Blocks of 32; a round pairs the nblk blocks by
// the round-robin (circle) schedule, so a sweep of nblk-1 rounds meets every
// block pair once.  A rotation (p, q) is applied only when
// |c_pq| > tol * sqrt(c_pp c_qq) (C is positive definite); a sweep without any
// such rotation ends the iteration.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rr_pos(int k, int r, int m) {
  return k == 0 ? 0 : 1 + ((k - 1 + r) % (m - 1));
}
__device__ __forceinline__ void pair_blocks(int i, int r, int nblk, int& x, int& y) {
  int a = rr_pos(i, r, nblk), b = rr_pos(nblk - 1 - i, r, nblk);
  x = a < b ? a : b;
  y = a < b ? b : a;
}

constexpr int JS = 2 * JB;      // subproblem size
constexpr int LDJ = JS + 1;
constexpr double kJacTol = 1e-14;      // relative to the pivots
constexpr double kJacAbs = 1e-13;      // relative to the largest diagonal entry
#ifndef KP_JAC_INNER
#define KP_JAC_INNER 1                   // inner sweeps per block-pair subproblem
#endif

// Jacobi rotation (c, s) that annihilates apq in [[app, apq], [apq, aqq]]
// (Golub & Van Loan, Alg. 8.4.1): theta = (aqq - app) / (2 apq),
// t = sign(theta) / (|theta| + sqrt(theta^2 + 1)), c = 1 / sqrt(1 + t^2), s = t c.
// The reciprocals and inverse square roots start from the hardware estimates
// and take Newton steps (each doubles the correct bits) to full precision; this
// shortens the dependent chain that every round of the sweep waits for.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int i = 0; i < 3; i++) y = fma(y, fma(-x, y, 1.0), y);   // y (2 - x y)
  return y;
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 3; i++) y = y * fma(-0.5 * x * y, y, 1.5);   // y (3 - x y^2) / 2
  return y;
}
__device__ __forceinline__ void rotation(double app, double aqq, double apq, double& c,
                                         double& s) {
  if (!(fabs(apq) > 1e-150)) {   // outside the estimates' range: plain divisions
    const double th = (aqq - app) / (2.0 * apq);
    const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
    c = 1.0 / sqrt(t * t + 1.0);
    s = t * c;
    return;
  }
  const double th = (aqq - app) * rcp_nr(2.0 * apq);
  if (!(fabs(th) < 1e150)) {   // theta^2 would overflow: t = 1 / (2 theta)
    c = 1.0;
    s = 0.5 * rcp_nr(th);
    return;
  }
  const double u = fma(th, th, 1.0);
  const double su = u * rsqrt_nr(u);   // sqrt(theta^2 + 1)
  const double t = copysign(rcp_nr(fabs(th) + su), th);
  c = rsqrt_nr(fma(t, t, 1.0));
  s = t * c;
}

constexpr int kSolveThreads = 512;

// S <- J^T S J on one 2x2 group: rows (ia, ib) rotated by (c1, s1), columns
// (jf, jg) by (c2, s2); x = S[ia][jf], S[ia][jg], S[ib][jf], S[ib][jg].
__device__ __forceinline__ void rot2x2(const double (&x)[4], double c1, double s1, double c2,
                                       double s2, double (&o)[4]) {
  const double raf = c1 * x[0] - s1 * x[2];
  const double rag = c1 * x[1] - s1 * x[3];
  const double rbf = s1 * x[0] + c1 * x[2];
  const double rbg = s1 * x[1] + c1 * x[3];
  o[0] = c2 * raf - s2 * rag;
  o[1] = s2 * raf + c2 * rag;
  o[2] = c2 * rbf - s2 * rbg;
  o[3] = s2 * rbf + c2 * rbg;
}

__device__ __forceinline__ void jac_rotation(double app, double aqq, double apq, double floor_abs,
                                             double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (fabs(apq) > fmax(kJacTol * sqrt(fabs(app * aqq)), floor_abs)) rotation(app, aqq, apq, c, s);
}

// The JB rounds across the two blocks of a subproblem: rotation k of round rr
// pairs k with JB + (k + rr) mod JB.  One barrier per round: thread k < JB owns
// the 2x2 groups (k, k) and (k, k + 1) and also recomputes (k + 1, k + 1), which
// hold the three entries that rotation k of the next round needs (pair k of
// round rr + 1 is (a_k, b_{k+1}) of round rr), so it computes that rotation
// right after its update.  The other threads take the groups (kx, kx + d),
// d = 2 .. JB - 1; V <- V J as in the first round.
__device__ void jac_cross_rounds(double* S, double* V, double2 (*rotx)[JB], int inner,
                                 double floor_abs) {
  const int t = threadIdx.x;
  auto pr_of = [](int k, int rr) { return make_int2(k, JB + ((k + rr) & (JB - 1))); };
  constexpr int VG = JB * JS / kSolveThreads;
  for (int sw = 0; sw < inner; sw++) {
    if (t < JB) {
      double c, s;
      jac_rotation(S[t * LDJ + t], S[(JB + t) * LDJ + JB + t], S[t * LDJ + JB + t], floor_abs, c, s);
      rotx[0][t] = make_double2(c, s);
    }
    __syncthreads();
    for (int rr = 0; rr < JB; rr++) {
      const int par = rr & 1;
      // V element pairs (loads first, as below)
      double y[VG][2], vc[VG], vs[VG];
      int va[VG], vb[VG], vr[VG];
#pragma unroll
      for (int it = 0; it < VG; it++) {
        const int e = t + it * kSolveThreads;
        const int k = e / JS;
        const int2 pk = pr_of(k, rr);
        const double2 rk = rotx[par][k];
        vr[it] = e % JS; va[it] = pk.x; vb[it] = pk.y; vc[it] = rk.x; vs[it] = rk.y;
        y[it][0] = V[vr[it] * LDJ + va[it]];
        y[it][1] = V[vr[it] * LDJ + vb[it]];
      }
      if (t < JB) {
        const int k = t, k1 = (t + 1) & (JB - 1);
        const int2 p0 = pr_of(k, rr), p1 = pr_of(k1, rr);
        const double2 r0 = rotx[par][k], r1 = rotx[par][k1];
        double g1[4], g2[4], g3[4];
        g1[0] = S[p0.x * LDJ + p0.x]; g1[1] = S[p0.x * LDJ + p0.y];
        g1[2] = S[p0.y * LDJ + p0.x]; g1[3] = S[p0.y * LDJ + p0.y];
        g2[0] = S[p0.x * LDJ + p1.x]; g2[1] = S[p0.x * LDJ + p1.y];
        g2[2] = S[p0.y * LDJ + p1.x]; g2[3] = S[p0.y * LDJ + p1.y];
        g3[0] = S[p1.x * LDJ + p1.x]; g3[1] = S[p1.x * LDJ + p1.y];
        g3[2] = S[p1.y * LDJ + p1.x]; g3[3] = S[p1.y * LDJ + p1.y];
        double n1[4], n2[4], n3[4];
        rot2x2(g1, r0.x, r0.y, r0.x, r0.y, n1);
        rot2x2(g2, r0.x, r0.y, r1.x, r1.y, n2);
        rot2x2(g3, r1.x, r1.y, r1.x, r1.y, n3);
        // (k1, k1) is written by thread k1 of this wave after this thread's reads
        S[p0.x * LDJ + p0.x] = n1[0]; S[p0.x * LDJ + p0.y] = n1[1];
        S[p0.y * LDJ + p0.x] = n1[2]; S[p0.y * LDJ + p0.y] = n1[3];
        S[p0.x * LDJ + p1.x] = n2[0]; S[p0.x * LDJ + p1.y] = n2[1];
        S[p0.y * LDJ + p1.x] = n2[2]; S[p0.y * LDJ + p1.y] = n2[3];
        if (rr + 1 < JB) {
          // next pair k = (a_k, b_{k1}): S'[a_k][a_k], S'[b_k1][b_k1], S'[a_k][b_k1]
          double c, s;
          jac_rotation(n1[0], n3[3], n2[1], floor_abs, c, s);
          rotx[par ^ 1][k] = make_double2(c, s);
        }
      } else {
        constexpr int NO = JB - 2;   // off-diagonal distances per row of groups
        double x[2][4];
        int ia[2], ib[2], jf[2], jg[2];
        double c1[2], s1[2], c2[2], s2[2];
#pragma unroll
        for (int it = 0; it < 2; it++) {
          const int g = (t - JB) + it * (kSolveThreads - JB);
          const int kx = g / NO, ky = (kx + 2 + g % NO) & (JB - 1);
          const int2 px = pr_of(kx, rr), py = pr_of(ky, rr);
          const double2 rx = rotx[par][kx], ry = rotx[par][ky];
          ia[it] = px.x; ib[it] = px.y; jf[it] = py.x; jg[it] = py.y;
          c1[it] = rx.x; s1[it] = rx.y; c2[it] = ry.x; s2[it] = ry.y;
          x[it][0] = S[ia[it] * LDJ + jf[it]];
          x[it][1] = S[ia[it] * LDJ + jg[it]];
          x[it][2] = S[ib[it] * LDJ + jf[it]];
          x[it][3] = S[ib[it] * LDJ + jg[it]];
        }
#pragma unroll
        for (int it = 0; it < 2; it++) {
          double o[4];
          rot2x2(x[it], c1[it], s1[it], c2[it], s2[it], o);
          S[ia[it] * LDJ + jf[it]] = o[0];
          S[ia[it] * LDJ + jg[it]] = o[1];
          S[ib[it] * LDJ + jf[it]] = o[2];
          S[ib[it] * LDJ + jg[it]] = o[3];
        }
      }
#pragma unroll
      for (int it = 0; it < VG; it++) {
        V[vr[it] * LDJ + va[it]] = vc[it] * y[it][0] - vs[it] * y[it][1];
        V[vr[it] * LDJ + vb[it]] = vs[it] * y[it][0] + vc[it] * y[it][1];
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kSolveThreads) void k_jac_solve(const EigProblem* __restrict__ pr,
                                                   const int* __restrict__ ids,
                                                   const int* __restrict__ done, int r,
                                                   int inner) {
  const int q = ids[blockIdx.y];
  const EigProblem p = pr[q];
  const int nblk = p.n_pad / JB;
  if (done[2 * q] || r >= nblk - 1) return;
  const int i = blockIdx.x;
  if (i >= nblk / 2) return;
  int bx, by;
  pair_blocks(i, r, nblk, bx, by);
  __shared__ double S[JS * LDJ];
  __shared__ double V[JS * LDJ];
  // rotation k of the round: (c, s) and its index pair (p, q), each read as one
  // 16- or 8-byte access
  __shared__ double2 rot[JB];
  __shared__ int2 pq[JB];
  __shared__ double2 rotx[2][JB];   // cross rounds: rotations by round parity
  __shared__ int any;
  const long np = p.n_pad;
  const double* C = p.C[0];
  if (threadIdx.x == 0) any = 0;
  const double floor_abs = kJacAbs * *p.dmax;
  for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
    const int a = e / JS, b = e % JS;
    const int ga = (a < JB ? bx * JB + a : by * JB + a - JB);
    const int gb = (b < JB ? bx * JB + b : by * JB + b - JB);
    S[a * LDJ + b] = C[(long)ga * np + gb];
    V[a * LDJ + b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) {
    const int a = e / JS, b = e % JS;
    if (a < b && fabs(S[a * LDJ + b]) >
                     fmax(kJacTol * sqrt(fabs(S[a * LDJ + a] * S[b * LDJ + b])), floor_abs))
      any = 1;
  }
  __syncthreads();
  if (!any) {
    if (threadIdx.x == 0) p.pflag[i] = 1;
    return;
  }
  // The first round of an outer sweep pairs every block once: its subproblems
  // take every index pair of the two blocks (2 JB - 1 rounds), so each pair
  // inside a block is met once per outer sweep.  The other rounds take only the
  // JB x JB pairs across the two blocks (JB rounds of JB disjoint pairs).
  const bool full = r == 0;
  const int nrr = full ? JS - 1 : JB;
  int rr = 0;
  // index pair of rotation k in round rr: from the table in the first round, by
  // formula in the others
  auto pair_of = [&](int k) -> int2 {
    if (full) return pq[k];
    return make_int2(k, JB + ((k + rr) & (JB - 1)));
  };
  if (!full) {
    jac_cross_rounds(S, V, rotx, inner, floor_abs);
  } else
  for (int sw = 0; sw < inner; sw++) {
    for (rr = 0; rr < nrr; rr++) {
      if (threadIdx.x < JB) {
        const int k = threadIdx.x;
        int a, b;
        if (full) {
          a = rr_pos(k, rr, JS);
          b = rr_pos(JS - 1 - k, rr, JS);
          if (a > b) { int t = a; a = b; b = t; }
        } else {
          a = k;
          b = JB + ((k + rr) & (JB - 1));
        }
        const double apq = S[a * LDJ + b], app = S[a * LDJ + a], aqq = S[b * LDJ + b];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > fmax(kJacTol * sqrt(fabs(app * aqq)), floor_abs)) rotation(app, aqq, apq, c, s);
        rot[k] = make_double2(c, s);
        pq[k] = make_int2(a, b);
      }
      __syncthreads();
      // S <- J^T S J on 2x2 groups (rows of pair kx, columns of pair ky), V <- V J.
      // The groups (and the V element pairs) are disjoint, so each thread loads
      // all of its operands before computing and storing: the LDS latency is paid
      // once per phase instead of once per element.
      constexpr int SG = JB * JB / kSolveThreads, VG = JB * JS / kSolveThreads;
      {
        double x[SG][4];
        int ia[SG], ib[SG], jf[SG], jg[SG];
        double c1[SG], s1[SG], c2[SG], s2[SG];
#pragma unroll
        for (int it = 0; it < SG; it++) {
          const int e = threadIdx.x + it * kSolveThreads;
          const int kx = e / JB, ky = e % JB;
          const int2 px = pair_of(kx), py = pair_of(ky);
          const double2 rx = rot[kx], ry = rot[ky];
          ia[it] = px.x; ib[it] = px.y; jf[it] = py.x; jg[it] = py.y;
          c1[it] = rx.x; s1[it] = rx.y; c2[it] = ry.x; s2[it] = ry.y;
          x[it][0] = S[ia[it] * LDJ + jf[it]];
          x[it][1] = S[ia[it] * LDJ + jg[it]];
          x[it][2] = S[ib[it] * LDJ + jf[it]];
          x[it][3] = S[ib[it] * LDJ + jg[it]];
        }
        double y[VG][2];
        int va[VG], vb[VG], vr[VG];
        double vc[VG], vs[VG];
#pragma unroll
        for (int it = 0; it < VG; it++) {
          const int e = threadIdx.x + it * kSolveThreads;
          const int k = e / JS;
          const int2 pk = pair_of(k);
          const double2 rk = rot[k];
          vr[it] = e % JS; va[it] = pk.x; vb[it] = pk.y; vc[it] = rk.x; vs[it] = rk.y;
          y[it][0] = V[vr[it] * LDJ + va[it]];
          y[it][1] = V[vr[it] * LDJ + vb[it]];
        }
#pragma unroll
        for (int it = 0; it < SG; it++) {
          const double raf = c1[it] * x[it][0] - s1[it] * x[it][2];
          const double rag = c1[it] * x[it][1] - s1[it] * x[it][3];
          const double rbf = s1[it] * x[it][0] + c1[it] * x[it][2];
          const double rbg = s1[it] * x[it][1] + c1[it] * x[it][3];
          S[ia[it] * LDJ + jf[it]] = c2[it] * raf - s2[it] * rag;
          S[ia[it] * LDJ + jg[it]] = s2[it] * raf + c2[it] * rag;
          S[ib[it] * LDJ + jf[it]] = c2[it] * rbf - s2[it] * rbg;
          S[ib[it] * LDJ + jg[it]] = s2[it] * rbf + c2[it] * rbg;
        }
#pragma unroll
        for (int it = 0; it < VG; it++) {
          V[vr[it] * LDJ + va[it]] = vc[it] * y[it][0] - vs[it] * y[it][1];
          V[vr[it] * LDJ + vb[it]] = vs[it] * y[it][0] + vc[it] * y[it][1];
        }
      }
      __syncthreads();
    }
  }
  double* Vo = p.V + (long)i * JS * JS;
  for (int e = threadIdx.x; e < JS * JS; e += blockDim.x) Vo[e] = V[(e / JS) * LDJ + (e % JS)];
  if (threadIdx.x == 0) {
    p.pflag[i] = 0;
    atomicOr(&p.pflag[p.n_pad / 64], 1);
  }
}

// pair index of block X in round r
__device__ __forceinline__ int block_pair_index(int X, int r, int nblk) {
  for (int i = 0; i < nblk / 2; i++) {
    int a, b;
    pair_blocks(i, r, nblk, a, b);
    if (a == X || b == X) return i;
  }
  return 0;
}

__device__ __forceinline__ long grow(int a, int b0, int b1) {
  return a < JB ? (long)b0 * JB + a : (long)b1 * JB + a - JB;
}

// In place: C region (pair X rows, pair Y cols) <- V_X^T C V_Y for pX <= pY
// (mirrored), then P[R rows, pair Y cols] <- P V_Y.  Identity pairs are skipped.
// Two LDS tiles, so two workgroups share a CU.
__global__ __launch_bounds__(256) void k_jac_apply(const EigProblem* __restrict__ pr,
                                                   const int* __restrict__ ids,
                                                   const int* __restrict__ done, int r) {
  const int q = ids[blockIdx.y];
  const EigProblem p = pr[q];
  const int nblk = p.n_pad / JB;
  if (done[2 * q] || r >= nblk - 1) return;
  const int npair = nblk / 2;
  const int ncg = npair * (npair + 1) / 2;
  int w = blockIdx.x;
  if (w >= ncg + npair * npair) return;
  const long np = p.n_pad;
  __shared__ double G[BB * LDM];
  __shared__ double W[BB * LDM];
  f64x4 acc[2][2];
  if (w < ncg) {
    int pX = 0, rowlen = npair;
    while (w >= rowlen) { w -= rowlen; pX++; rowlen--; }
    const int pY = pX + w;
    const bool ix = p.pflag[pX] != 0, iy = p.pflag[pY] != 0;
    if (ix && iy) return;
    int x0, x1, y0, y1;
    pair_blocks(pX, r, nblk, x0, x1);
    pair_blocks(pY, r, nblk, y0, y1);
    double* C = p.C[0];
    for (int e = threadIdx.x; e < BB * BB; e += blockDim.x) {
      const int a = e / BB, b = e % BB;
      G[a * LDM + b] = C[grow(a, x0, x1) * np + grow(b, y0, y1)];
      W[a * LDM + b] = iy ? p.V[(long)pX * BB * BB + e] : p.V[(long)pY * BB * BB + e];
    }
    __syncthreads();
    auto store_c = [&](int i, int j, double v) {
      const long gr = grow(i, x0, x1), gc = grow(j, y0, y1);
      C[gr * np + gc] = v;
      if (pX != pY) C[gc * np + gr] = v;
    };
    if (!iy) {   // C V_Y
      mm64_zero(acc);
      mm64<false, false>(acc, G, W);
      if (ix) {   // V_X is the identity: done
        mm64_each(acc, store_c);
        return;
      }
      __syncthreads();
      mm64_each(acc, [&](int i, int j, double v) { G[i * LDM + j] = v; });
      for (int e = threadIdx.x; e < BB * BB; e += blockDim.x)
        W[(e / BB) * LDM + (e % BB)] = p.V[(long)pX * BB * BB + e];
      __syncthreads();
    }
    // V_X^T G (W holds V_X)
    mm64_zero(acc);
    mm64<true, false>(acc, W, G);
    mm64_each(acc, store_c);
  } else {
    w -= ncg;
    const int R = w / npair, pY = w % npair;
    if (p.pflag[pY]) return;
    int y0, y1;
    pair_blocks(pY, r, nblk, y0, y1);
    double* P = p.P[0];
    for (int e = threadIdx.x; e < BB * BB; e += blockDim.x) {
      const int a = e / BB, b = e % BB;
      G[a * LDM + b] = P[((long)R * BB + a) * np + grow(b, y0, y1)];
      W[a * LDM + b] = p.V[(long)pY * BB * BB + e];
    }
    __syncthreads();
    mm64_zero(acc);
    mm64<false, false>(acc, G, W);
    mm64_each(acc, [&](int i, int j, double v) { P[((long)R * BB + i) * np + grow(j, y0, y1)] = v; });
  }
}

// After a sweep: converged when no rotation exceeded the threshold.
__global__ void k_jac_check(const EigProblem* __restrict__ pr, const int* __restrict__ ids,
                            int* done, int nprob) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nprob) return;
  const int q = ids[i];
  const EigProblem p = pr[q];
  if (done[2 * q]) return;
  int* rot = &p.pflag[p.n_pad / 64];
  if (*rot == 0) done[2 * q] = 1;
  done[2 * q + 1] += 1;   // sweeps used
  *rot = 0;
}

// After the last scheduled sweep: a problem that still rotated in its last sweep
// has not converged; its e = diag(C) would not diagonalise the whitened factor, so
// the owning context's status becomes 7 (unless an earlier failure is recorded).
__global__ void k_jac_final(const EigProblem* __restrict__ pr, const int* __restrict__ done,
                            int nprob, int* status) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nprob || done[2 * q]) return;
  int* s = pr[q].status ? pr[q].status : status;
  atomicCAS(s, 0, 7);
}

__global__ void k_jac_extract(const EigProblem* __restrict__ pr) {
  const EigProblem p = pr[blockIdx.y];
  const long np = p.n_pad;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)p.n * p.n;
       e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / p.n), j = (int)(e % p.n);
    p.Pout[e] = p.P[1][(long)i * np + j];
    if (i == j) p.eout[i] = p.C[0][(long)i * np + i];
  }
}

hipError_t eig_host_sync(EigGroups& g, const int* ids, int nprob) {
  if (g.host) return hipSuccess;
  const size_t bytes = sizeof(int) * ((size_t)nprob + 4 * kEigGroups * (size_t)nprob);
  if (hipError_t e = hipHostMalloc((void**)&g.host, bytes, hipHostMallocDefault)) {
    g.host = nullptr;
    return e;
  }
  std::memcpy(g.host, ids, sizeof(int) * nprob);
  for (int k = 0; k < g.n; k++)
    for (int par = 0; par < 2; par++)
      if (hipError_t e = hipEventCreateWithFlags(&g.swept[k][par], hipEventDisableTiming)) {
        eig_host_free(g);
        return e;
      }
  g.host_nprob = nprob;
  return hipSuccess;
}

static void sweep_graphs_free(EigGroups& g) {
  for (int k = 0; k < kEigGroups; k++)
    for (int par = 0; par < 2; par++) {
      if (g.sweep[k][par]) (void)hipGraphExecDestroy(g.sweep[k][par]);
      if (g.sweep_graph[k][par]) (void)hipGraphDestroy(g.sweep_graph[k][par]);
      g.sweep[k][par] = nullptr;
      g.sweep_graph[k][par] = nullptr;
    }
  g.sweep_key[0] = g.sweep_key[1] = g.sweep_key[2] = nullptr;
}

void eig_host_free(EigGroups& g) {
  for (int k = 0; k < kEigGroups; k++)
    for (int par = 0; par < 2; par++)
      if (g.swept[k][par]) {
        (void)hipEventSynchronize(g.swept[k][par]);
        (void)hipEventDestroy(g.swept[k][par]);
        g.swept[k][par] = nullptr;
      }
  sweep_graphs_free(g);
  if (g.cap) (void)hipStreamDestroy(g.cap);
  g.cap = nullptr;
  if (g.host) (void)hipHostFree(g.host);
  g.host = nullptr;
  g.host_nprob = 0;
}

void eig_groups_plan(const EigProblem* probs, int nprob, int ngroups, int* ids, EigGroups& g) {
  ngroups = std::max(1, std::min(ngroups, std::min(nprob, kEigGroups)));
  // largest first, each to the group with the least work so far (work ~ n_pad^3)
  std::vector<int> order(nprob);
  for (int q = 0; q < nprob; q++) order[q] = q;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return probs[a].n_pad > probs[b].n_pad; });
  std::vector<std::vector<int>> mem(ngroups);
  std::vector<double> load(ngroups, 0.0);
  for (int q : order) {
    int k = 0;
    for (int j = 1; j < ngroups; j++)
      if (load[j] < load[k]) k = j;
    mem[k].push_back(q);
    load[k] += std::pow((double)probs[q].n_pad, 3.0);
  }
  g.n = ngroups;
  int o = 0;
  for (int k = 0; k < ngroups; k++) {
    g.off[k] = o;
    g.npmax[k] = 0;
    std::sort(mem[k].begin(), mem[k].end());
    for (int q : mem[k]) {
      ids[o++] = q;
      g.npmax[k] = std::max(g.npmax[k], probs[q].n_pad);
    }
  }
  g.off[ngroups] = o;
}

hipError_t kron_eig_batched(const EigProblem* probs_host, int nprob, double lambda,
                            EigProblem* probs_dev, int* status, int* done, int* calls,
                            int refresh, int max_sweeps, EigGroups& g, hipStream_t st) {
  if (nprob <= 0) return hipSuccess;
  if (g.n < 1 || g.n > kEigGroups || g.off[0] != 0 || g.off[g.n] != nprob || !g.ids)
    return hipErrorInvalidValue;
  int npmax = 0;
  for (int q = 0; q < nprob; q++) npmax = probs_host[q].n_pad > npmax ? probs_host[q].n_pad : npmax;
  const int nbmax = npmax / BB;
  k_eig_begin<<<1, 1, 0, st>>>(calls, refresh);
  k_damp_pad<<<dim3(256, nprob), 256, 0, st>>>(probs_dev, lambda);
  for (int j = 0; j < nbmax; j++) {
    k_chol_diag<<<dim3(1, nprob), 256, 0, st>>>(probs_dev, j, status);
    const int rem = nbmax - 1 - j;
    if (rem > 0) {
      const int nw = rem * (rem + 3) / 2;   // sum_{i=j+1}^{nb-1} (i - j + 1)
      k_chol_update<<<dim3(nw, nprob), 256, 0, st>>>(probs_dev, j);
    }
  }
  for (int i = 1; i < nbmax; i++) k_trtri_row<<<dim3(i, nprob), 256, 0, st>>>(probs_dev, i);
  const dim3 gmm(nbmax, nbmax, nprob);
  k_eig_mm<0><<<gmm, 256, 0, st>>>(probs_dev, calls + 1);
  k_eig_mm<1><<<gmm, 256, 0, st>>>(probs_dev, calls + 1);
  k_eig_mm<2><<<gmm, 256, 0, st>>>(probs_dev, calls + 1);
  k_eig_mm<3><<<gmm, 256, 0, st>>>(probs_dev, calls + 1);
  k_jac_init<<<dim3(256, nprob), 256, 0, st>>>(probs_dev, done, calls + 1);
  k_jac_dmax<<<nprob, 256, 0, st>>>(probs_dev);
  // Sweeps of the groups, interleaved round by round on their streams: the
  // rounds of one group form a dependent chain of short launches, so chains of
  // other groups fill the machine meanwhile.
  const int ng = g.n;
  if (ng > 1) {
    if (hipError_t e = hipEventRecord(g.fork, st)) return e;
    for (int k = 1; k < ng; k++)
      if (hipError_t e = hipStreamWaitEvent(g.st[k], g.fork, 0)) return e;
  }
  // Sweep by sweep; within a sweep the groups' rounds interleave launch by launch.
  int rounds[kEigGroups], rmax = 0;
  bool active[kEigGroups];
  for (int k = 0; k < ng; k++) {
    rounds[k] = g.npmax[k] / JB - 1;
    rmax = std::max(rmax, rounds[k]);
    active[k] = rounds[k] >= 1;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusActive;
  const bool early = g.host && g.host_wait && g.host_nprob == nprob && hipStreamIsCapturing(st, &cap) == hipSuccess &&
                     cap == hipStreamCaptureStatusNone;
  const long nflag = 2L * nprob;
  auto flags = [&](int k, int par) { return g.host + nprob + (2 * k + par) * nflag; };
  // one group's sweep: its rounds, the convergence check and (early stop) the copy
  // of the flags for the host
  auto enqueue_sweep = [&](int k, int par, hipStream_t sk) -> hipError_t {
    const int* ids = g.ids + g.off[k];
    const int nq = g.off[k + 1] - g.off[k];
    const int npair = g.npmax[k] / JB / 2;
    const int nwg = npair * (npair + 1) / 2 + npair * npair;
    for (int r = 0; r < rounds[k]; r++) {
      k_jac_solve<<<dim3(npair, nq), kSolveThreads, 0, sk>>>(probs_dev, ids, done, r, KP_JAC_INNER);
      k_jac_apply<<<dim3(nwg, nq), 256, 0, sk>>>(probs_dev, ids, done, r);
    }
    k_jac_check<<<(nq + 63) / 64, 64, 0, sk>>>(probs_dev, ids, done, nq);
    if (hipError_t e = hipGetLastError()) return e;
    if (!early) return hipSuccess;
    return hipMemcpyAsync(flags(k, par), done, sizeof(int) * nflag, hipMemcpyDeviceToHost, sk);
  };
  if (early && (g.sweep_key[0] != probs_dev || g.sweep_key[1] != done || g.sweep_key[2] != g.ids))
    sweep_graphs_free(g);
  // the early stop's sweeps as graphs (captured once on a private stream)
  auto sweep_graph = [&](int k, int par) -> hipGraphExec_t {
    if (g.sweep[k][par]) return g.sweep[k][par];
    if (!g.cap && hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking) != hipSuccess) {
      g.cap = nullptr;
      return nullptr;
    }
    if (hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    const hipError_t e = enqueue_sweep(k, par, g.cap);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(g.cap, &gr);
    if (e != hipSuccess || e2 != hipSuccess || !gr) {
      if (gr) (void)hipGraphDestroy(gr);
      return nullptr;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, gr, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(gr);
      return nullptr;
    }
    g.sweep_graph[k][par] = gr;
    g.sweep[k][par] = x;
    g.sweep_key[0] = probs_dev;
    g.sweep_key[1] = done;
    g.sweep_key[2] = g.ids;
    return x;
  };
  for (int sw = 0; sw < max_sweeps; sw++) {
    bool any = false;
    for (int k = 0; k < ng; k++) any = any || active[k];
    if (!any) break;
    if (early) {
      for (int k = 0; k < ng; k++) {
        if (!active[k] || rounds[k] < 1) continue;
        const hipStream_t sk = k == 0 ? st : g.st[k];
        if (hipGraphExec_t x = sweep_graph(k, sw & 1)) {
          if (hipError_t e = hipGraphLaunch(x, sk)) return e;
        } else if (hipError_t e = enqueue_sweep(k, sw & 1, sk)) {
          return e;
        }
        if (hipError_t e = hipEventRecord(g.swept[k][sw & 1], sk)) return e;
      }
    } else {
      // the groups' rounds interleaved launch by launch on their streams
      for (int r = 0; r < rmax; r++)
        for (int k = 0; k < ng; k++) {
          if (!active[k] || r >= rounds[k]) continue;
          const hipStream_t sk = k == 0 ? st : g.st[k];
          const int* ids = g.ids + g.off[k];
          const int nq = g.off[k + 1] - g.off[k];
          const int npair = g.npmax[k] / JB / 2;
          const int nwg = npair * (npair + 1) / 2 + npair * npair;
          k_jac_solve<<<dim3(npair, nq), kSolveThreads, 0, sk>>>(probs_dev, ids, done, r, KP_JAC_INNER);
          k_jac_apply<<<dim3(nwg, nq), 256, 0, sk>>>(probs_dev, ids, done, r);
          if (r < rounds[k] - 1) continue;
          k_jac_check<<<(nq + 63) / 64, 64, 0, sk>>>(probs_dev, ids, done, nq);
        }
    }
    if (!early || sw == 0) continue;
    // the previous sweep's flags (this sweep is already queued behind it)
    for (int k = 0; k < ng; k++) {
      if (!active[k]) continue;
      if (hipError_t e = hipEventSynchronize(g.swept[k][(sw - 1) & 1])) return e;
      const int* f = flags(k, (sw - 1) & 1);
      bool all = true;
      for (int i = g.off[k]; i < g.off[k + 1] && all; i++) all = f[2 * g.host[i]] != 0;
      if (all) active[k] = false;
    }
  }
  if (ng > 1) {
    for (int k = 1; k < ng; k++) {
      if (hipError_t e = hipEventRecord(g.join[k], g.st[k])) return e;
      if (hipError_t e = hipStreamWaitEvent(st, g.join[k], 0)) return e;
    }
  }
  k_jac_final<<<(nprob + 63) / 64, 64, 0, st>>>(probs_dev, done, nprob, status);
  k_eig_mm<4><<<gmm, 256, 0, st>>>(probs_dev, calls + 1);
  k_jac_extract<<<dim3(64, nprob), 256, 0, st>>>(probs_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Kronecker-sum apply (per layer, FP64):
//   Delta = -P_B [(P_B^T V P_A) / (1 + b a^T)] P_A^T
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gemm64_tile(const G64& g) {
  const int i0 = blockIdx.y * BB, j0 = blockIdx.x * BB;
  if (i0 >= g.M || j0 >= g.N) return;
  __shared__ __align__(16) double As[BB * LDM];
  __shared__ __align__(16) double Bs[BB * LDM];
  f64x4 acc[2][2];
  mm64_zero(acc);
  for (int k0 = 0; k0 < g.K; k0 += BB) {
    __syncthreads();
    for (int e = threadIdx.x; e < BB * BB; e += blockDim.x) {
      const int a = e / BB, b = e % BB;
      As[a * LDM + b] = (i0 + a < g.M && k0 + b < g.K) ? g.A[(i0 + a) * g.sai + (k0 + b) * g.sak] : 0.0;
      Bs[a * LDM + b] = (k0 + a < g.K && j0 + b < g.N) ? g.B[(k0 + a) * g.sbk + (j0 + b) * g.sbj] : 0.0;
    }
    __syncthreads();
    mm64<false, false>(acc, As, Bs);
  }
  mm64_each(acc, [&](int a, int b, double v) {
    const int i = i0 + a, j = j0 + b;
    if (i < g.M && j < g.N) {
      v *= g.alpha;
      if (g.ea) v /= (1.0 + g.eb[i] * g.ea[j]);
      g.C[i * g.sci + j * g.scj] = v;
    }
  });
}

// descriptors in device memory, one product per grid.z
__global__ __launch_bounds__(256) void k_gemm64(const G64* __restrict__ gs) {
  gemm64_tile(gs[blockIdx.z]);
}

// one product whose descriptor travels as the kernel argument
__global__ __launch_bounds__(256) void k_gemm64_arg(const G64 g) { gemm64_tile(g); }

hipError_t gemm64_one(const G64& g, hipStream_t st) {
  k_gemm64_arg<<<dim3(kp_cdiv(g.N, BB), kp_cdiv(g.M, BB), 1), 256, 0, st>>>(g);
  return hipGetLastError();
}

void kron_apply_descs(const KronApply* layers, int L, const double* grad, double* delta,
                      double* tmp, long tmp_stride, G64* h, int* mmax, int* nmax) {
  *mmax = 0;
  *nmax = 0;
  for (int l = 0; l < L; l++) {
    const KronApply& k = layers[l];
    double* T1 = tmp + (long)l * tmp_stride;             // nB x nA
    double* T2 = T1 + (long)k.nA * k.nB;                 // nB x nA
    const double* V = grad + k.off;                      // V[i][j] at j*nB + i
    double* D = delta + k.off;
    // T1 = P_B^T V
    h[0 * L + l] = G64{k.PB, 1, k.nB, V, 1, k.nB, T1, k.nA, 1, k.nB, k.nA, k.nB, 1.0, nullptr, nullptr};
    // T2 = (T1 P_A) / (1 + b a^T)
    h[1 * L + l] = G64{T1, k.nA, 1, k.PA, k.nA, 1, T2, k.nA, 1, k.nB, k.nA, k.nA, 1.0, k.a, k.b};
    // T1 = P_B T2
    h[2 * L + l] = G64{k.PB, k.nB, 1, T2, k.nA, 1, T1, k.nA, 1, k.nB, k.nA, k.nB, 1.0, nullptr, nullptr};
    // D = -T1 P_A^T  (column-major into the theta layout)
    h[3 * L + l] = G64{T1, k.nA, 1, k.PA, 1, k.nA, D, 1, k.nB, k.nB, k.nA, k.nA, -1.0, nullptr, nullptr};
    *mmax = k.nB > *mmax ? k.nB : *mmax;
    *nmax = k.nA > *nmax ? k.nA : *nmax;
  }
}

hipError_t kron_apply_batched(const G64* descs_dev, int L, int mmax, int nmax, hipStream_t st) {
  dim3 g(kp_cdiv(nmax, BB), kp_cdiv(mmax, BB), L);
  for (int s = 0; s < 4; s++) k_gemm64<<<g, 256, 0, st>>>(descs_dev + s * L);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The same apply for one layer without any allocation: the two nB x nA
// intermediate products live in `scratch`, a file-scope device array (one copy
// per GPU, held until the process ends), and the four product descriptors are
// kernel arguments.  Host code never passes `scratch` itself to a kernel: its
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[2 * kKronScratchElems];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};
}  // namespace

static hipError_t scratch_address(double** out) {
  int dev = -1;
  if (hipError_t e = hipGetDevice(&dev)) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = (double*)p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

hipError_t kron_apply_noalloc(const KronApply& layer, const double* grad, double* delta,
                              hipStream_t st) {
  if ((long)layer.nA * layer.nB > kKronScratchElems) return hipErrorInvalidValue;
  double* tmp = nullptr;
  if (hipError_t e = scratch_address(&tmp)) return e;
  KronApply k = layer;
  k.off = 0;
  G64 h[4];
  int mmax = 0, nmax = 0;
  kron_apply_descs(&k, 1, grad, delta, tmp, 2L * k.nA * k.nB, h, &mmax, &nmax);
  const dim3 g(kp_cdiv(nmax, BB), kp_cdiv(mmax, BB), 1);
  for (int s = 0; s < 4; s++) k_gemm64_arg<<<g, 256, 0, st>>>(h[s]);
  return hipGetLastError();
}

}  // namespace kp
