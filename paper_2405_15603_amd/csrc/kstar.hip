// KFAC* (Section 3.4, paragraph "Learning rate and momentum"): the automatic
// learning rate and momentum of the quadratic model with the exact damped Gramian.
//
// The Gramian enters through d_i^T G d_j = (1/N) sum_n (J_n d_i)(J_n d_j) + the
// boundary term, so one Jacobian-vector product per direction suffices.  The
// residual of point n depends on layer l's parameters only through the layer
// outputs Z^(l)_{n,s} = W~^(l) z~^(l-1)_{n,s} of its shared rows s (Section 3.2),
// so the chain rule gives the JVP from the slabs the curvature pass already
// stored: J_n d = sum_l sum_s g^(l)_{n,s}^T D^(l) z~^(l-1)_{n,s}, with g the
// output gradients of the backward pass and D^(l) the direction's layer block.
// No extra forward pass is needed.
//
// The same slabs give the exact Gramian block of a layer (Section 3.2,
// Eq. laplace_gramian_block_exact): J_n = sum_s z~_{n,s} (x) g_{n,s} per point,
// then G = J^T J / N.
#include <algorithm>

#include "common.h"
#include "launch.h"

namespace kp {

namespace {
constexpr int JT = 64;   // slab rows and output columns per tile
constexpr int JK = 16;   // input columns per stage
}  // namespace

// part[(dir * ntj + jt) * R + row] = sum_{j in tile jt} G[row][j] (Z~ D_dir^T)[row][j]
// for dir 0 (D from d0, double) and dir 1 (D from d1, the slab type).  D_dir is
// the layer block of a direction in the theta layout: column-major H x K.
// Block: 64 rows x 64 output columns; thread (ty, tx) owns rows 4 ty .. 4 ty + 3
// and columns 4 tx .. 4 tx + 3; the 16 threads of a row group are consecutive
// lanes of one wavefront and reduce over their columns with lane shuffles.
template <typename T>
__global__ __launch_bounds__(256) void k_jvp_rows(const T* __restrict__ Z, long ldz,
                                                  const T* __restrict__ G, long ldg, int R, int K,
                                                  int H, const double* __restrict__ d0,
                                                  const T* __restrict__ d1, T* __restrict__ part) {
  __shared__ T Zs[JK][JT + 4];
  __shared__ T Ds[2][JK][JT + 4];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  const long r0 = (long)blockIdx.x * JT;
  const int j0 = blockIdx.y * JT;
  T acc[2][4][4];
#pragma unroll
  for (int d = 0; d < 2; d++)
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int c = 0; c < 4; c++) acc[d][i][c] = T(0);
  const int zr = tid >> 2, zk = (tid & 3) * 4;   // Z tile loader: 4 input columns of a row
  for (int k0 = 0; k0 < K; k0 += JK) {
    {
      const long row = r0 + zr;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int k = k0 + zk + e;
        Zs[zk + e][zr] = (row < R && k < K) ? Z[row * ldz + k] : T(0);
      }
    }
    for (int e = tid; e < JK * JT; e += 256) {
      const int kk = e / JT, jj = e % JT;
      const int k = k0 + kk, j = j0 + jj;
      const bool ok = k < K && j < H;
      Ds[0][kk][jj] = ok ? (T)d0[(long)k * H + j] : T(0);
      Ds[1][kk][jj] = ok ? d1[(long)k * H + j] : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < JK; kk++) {
      T a[4], b0[4], b1[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = Zs[kk][4 * ty + i];
#pragma unroll
      for (int c = 0; c < 4; c++) {
        b0[c] = Ds[0][kk][4 * tx + c];
        b1[c] = Ds[1][kk][4 * tx + c];
      }
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int c = 0; c < 4; c++) {
          acc[0][i][c] += a[i] * b0[c];
          acc[1][i][c] += a[i] * b1[c];
        }
    }
    __syncthreads();
  }
  const int ntj = gridDim.y;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const long row = r0 + 4 * ty + i;
    T s0 = T(0), s1 = T(0);
    if (row < R) {
#pragma unroll
      for (int c = 0; c < 4; c++) {
        const int j = j0 + 4 * tx + c;
        if (j < H) {
          const T gv = G[row * ldg + j];
          s0 += acc[0][i][c] * gv;
          s1 += acc[1][i][c] * gv;
        }
      }
    }
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) {
      s0 += __shfl_xor(s0, m, 64);
      s1 += __shfl_xor(s1, m, 64);
    }
    if (tx == 0 && row < R) {
      part[(long)blockIdx.y * R + row] = s0;
      part[(long)(ntj + blockIdx.y) * R + row] = s1;
    }
  }
}

// jv[dir * ldjv + n] (+)= sum_{jt < ntj} sum_{s < S} part[(dir * ntj + jt) * R + s * N + n]
// in FP64, in a fixed order (R = N * S, slab rows are s-major).
template <typename T>
__global__ void k_jvp_gather(const T* __restrict__ part, int ntj, int N, int S,
                             double* __restrict__ jv, long ldjv, int accumulate) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int dir = blockIdx.y;
  if (n >= N) return;
  const long R = (long)N * S;
  double v = 0.0;
  for (int jt = 0; jt < ntj; jt++) {
    const T* p = part + (long)(dir * ntj + jt) * R + n;
    for (int s = 0; s < S; s++) v += to_d(p[(long)s * N]);
  }
  double* o = jv + dir * ldjv + n;
  *o = accumulate ? *o + v : v;
}

int jvp_tiles(int h_out) { return kp_cdiv(h_out, JT); }

hipError_t jvp_layer(Prec p, const void* zin, long ldz, const void* g, long ldg, int n, int S,
                     int K, int H, const double* d0, const void* d1, void* part, double* jv,
                     long ldjv, int accumulate, hipStream_t st) {
  const long R = (long)n * S;
  if (R <= 0) return hipSuccess;
  const int ntj = jvp_tiles(H);
  dim3 grid(kp_cdiv(R, JT), ntj);
  dim3 gg(kp_cdiv(n, 256), 2);
  if (p == P_F64) {
    k_jvp_rows<double><<<grid, 256, 0, st>>>((const double*)zin, ldz, (const double*)g, ldg,
                                             (int)R, K, H, d0, (const double*)d1, (double*)part);
    k_jvp_gather<double><<<gg, 256, 0, st>>>((const double*)part, ntj, n, S, jv, ldjv, accumulate);
  } else if (p == P_F32) {
    k_jvp_rows<float><<<grid, 256, 0, st>>>((const float*)zin, ldz, (const float*)g, ldg, (int)R,
                                            K, H, d0, (const float*)d1, (float*)part);
    k_jvp_gather<float><<<gg, 256, 0, st>>>((const float*)part, ntj, n, S, jv, ldjv, accumulate);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// work[n * p + k * H + j] = sum_s Z[s N + n][k] G[s N + n][j]  (p = K H): the
// per-point Jacobian of the residual with respect to the layer's parameters in
// the theta layout (column-stacked [W | b], so entry (j, k) sits at k H + j).
template <typename T>
__global__ void k_layer_jac(const T* __restrict__ Z, long ldz, const T* __restrict__ G, long ldg,
                            int N, int S, int K, int H, double* __restrict__ work) {
  const long p = (long)K * H;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)N * p;
       e += (long)gridDim.x * blockDim.x) {
    const int n = (int)(e / p);
    const long q = e - (long)n * p;
    const int k = (int)(q / H), j = (int)(q - (long)k * H);
    double v = 0.0;
    for (int s = 0; s < S; s++) {
      const long row = (long)s * N + n;
      v += to_d(Z[row * ldz + k]) * to_d(G[row * ldg + j]);
    }
    work[e] = v;
  }
}

hipError_t layer_gramian(Prec p, const void* zin, long ldz, const void* g, long ldg, int n, int S,
                         int K, int H, double* work, double* out, hipStream_t st) {
  const long np = (long)K * H;
  const long tot = (long)n * np;
  const int nb = (int)std::min<long>(16384, (tot + 255) / 256);
  if (p == P_F64)
    k_layer_jac<double><<<nb, 256, 0, st>>>((const double*)zin, ldz, (const double*)g, ldg, n, S, K,
                                           H, work);
  else if (p == P_F32)
    k_layer_jac<float><<<nb, 256, 0, st>>>((const float*)zin, ldz, (const float*)g, ldg, n, S, K,
                                          H, work);
  else
    return hipErrorInvalidValue;
  if (hipError_t e = hipGetLastError()) return e;
  // out = J^T J / n on the FP64 matrix unit: A(i, k) = J[k][i], B(k, j) = J[k][j]
  G64 d{work, 1, np, work, np, 1, out, np, 1, (int)np, (int)np, n, 1.0 / n, nullptr, nullptr};
  return gemm64_one(d, st);
}

// ---------------------------------------------------------------------------
// The 2 x 2 model and the update, in one workgroup (deterministic reductions):
//   q11 = |J Delta|^2/N + |J_b Delta|^2/M + lambda |Delta|^2
//   q12 = <J Delta, J delta>/N + <J_b Delta, J_b delta>/M + lambda <Delta, delta>
//   q22 = |J delta|^2/N + |J_b delta|^2/M + lambda |delta|^2
//   b = (<Delta, g>, <delta, g>);   (alpha, mu) = -Q^-1 b
// At the first step (step counter 0: no previous update) mu = 0 and
// alpha = -b1 / q11; likewise when Q is numerically singular (delta parallel
// to Delta).
// ---------------------------------------------------------------------------
struct StepInfoK {
  double loss_interior, loss_boundary, lr_chosen, loss_after;
  int status, step;
  double momentum_chosen;
};

template <typename TP>
__global__ __launch_bounds__(1024) void k_kstar_solve(
    const double* __restrict__ jvi, long ldi, int N, const double* __restrict__ jvb, long ldb,
    int M, const double* __restrict__ Delta, const TP* __restrict__ delta,
    const double* __restrict__ grad, long D, double lambda, const double* __restrict__ base,
    int* status, int* step, double* coef, StepInfoK* info) {
  __shared__ double red[11][16];
  // point sums: 0 |J Delta|^2, 1 <J Delta, J delta>, 2 |J delta|^2 over the interior
  // points; 3..5 the same over the boundary points
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const double a = jvi[n], b = jvi[ldi + n];
    s[0] += a * a;
    s[1] += a * b;
    s[2] += b * b;
  }
  for (int n = threadIdx.x; n < M; n += blockDim.x) {
    const double a = jvb[n], b = jvb[ldb + n];
    s[3] += a * a;
    s[4] += a * b;
    s[5] += b * b;
  }
  double p[5] = {0, 0, 0, 0, 0};   // |D|^2, <D,d>, |d|^2, <D,g>, <d,g>
  for (long e = threadIdx.x; e < D; e += blockDim.x) {
    const double x = Delta[e], y = (double)delta[e], gv = grad[e];
    p[0] += x * x;
    p[1] += x * y;
    p[2] += y * y;
    p[3] += x * gv;
    p[4] += y * gv;
  }
  const double all[11] = {s[0], s[1], s[2], s[3], s[4], s[5], p[0], p[1], p[2], p[3], p[4]};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 11; q++) {
    const double v = warp_sum(all[q]);
    if (lane == 0) red[q][wave] = v;
  }
  __syncthreads();
  double tot[11];
  if (threadIdx.x == 0)
    for (int q = 0; q < 11; q++) {
      double t = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += red[q][w];
      tot[q] = t;
    }
  if (threadIdx.x != 0) return;
  const double iN = N > 0 ? 1.0 / N : 0.0, iM = M > 0 ? 1.0 / M : 0.0;
  const double q11 = tot[0] * iN + tot[3] * iM + lambda * tot[6];
  const double q12 = tot[1] * iN + tot[4] * iM + lambda * tot[7];
  const double q22 = tot[2] * iN + tot[5] * iM + lambda * tot[8];
  const double b1 = tot[9], b2 = tot[10];
  double a = 0.0, mu = 0.0;
  int st = *status;
  if (!isfinite(base[0]) || !isfinite(base[1])) st = 5;
  if (st == 0) {
    const double det = q11 * q22 - q12 * q12;
    if (*step == 0 || !(det > 1e-14 * q11 * q22)) {
      a = -b1 / q11;
    } else {
      a = -(q22 * b1 - q12 * b2) / det;
      mu = -(q11 * b2 - q12 * b1) / det;
    }
    if (!isfinite(a) || !isfinite(mu)) st = 5;
  }
  if (st != 0) a = mu = 0.0;
  *status = st;
  coef[0] = a;
  coef[1] = mu;
  if (st == 0) *step += 1;
  if (info) {
    info->loss_interior = base[0];
    info->loss_boundary = base[1];
    info->lr_chosen = a;
    info->loss_after = __builtin_nan("");
    info->status = st;
    info->step = *step;
    info->momentum_chosen = mu;
  }
}

template <typename TP>
__global__ void k_kstar_update(const int* __restrict__ status, const double* __restrict__ coef,
                               const double* __restrict__ Delta, TP* __restrict__ delta,
                               TP* __restrict__ theta, long D) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D || *status != 0) return;
  const TP d = (TP)(coef[0] * Delta[e] + coef[1] * (double)delta[e]);
  delta[e] = d;
  theta[e] = theta[e] + d;
}

hipError_t kstar_finish(Prec p, const double* jvi, long ldi, int N, const double* jvb, long ldb,
                        int M, const double* Delta, void* delta, const double* grad, long D,
                        double lambda, const double* base_loss, int* status, int* step,
                        void* theta, void* info, hipStream_t st) {
  double* coef = (double*)(status + 4);   // alpha, mu: the scalar slots after the status word
  const int nb = kp_cdiv(D, 256);
  if (p == P_F64) {
    k_kstar_solve<double><<<1, 1024, 0, st>>>(jvi, ldi, N, jvb, ldb, M, Delta,
                                              (const double*)delta, grad, D, lambda, base_loss,
                                              status, step, coef, (StepInfoK*)info);
    k_kstar_update<double><<<nb, 256, 0, st>>>(status, coef, Delta, (double*)delta,
                                               (double*)theta, D);
  } else {
    k_kstar_solve<float><<<1, 1024, 0, st>>>(jvi, ldi, N, jvb, ldb, M, Delta,
                                             (const float*)delta, grad, D, lambda, base_loss,
                                             status, step, coef, (StepInfoK*)info);
    k_kstar_update<float><<<nb, 256, 0, st>>>(status, coef, Delta, (float*)delta, (float*)theta,
                                              D);
  }
  return hipGetLastError();
}

}  // namespace kp
