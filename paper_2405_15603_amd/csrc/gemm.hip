// Dense products of the hot path, on the 16x16 MFMA tiles of gfx950.
//
//  * gemm_nt: the layer products of the forward Laplacian (T_out = W~ T~_in per
//    slab row, Eq. forward-laplacian-linear-layer-compact) and of its backward
//    pass (Tbar_in = W^T Tbar_out).  Slab rows are the M dimension; both
//    operands keep K contiguous, so 16-byte global loads feed LDS directly.
//  * gemm_tn_splitk: the Kronecker factors (Eq. KFAC-PINN: sums of outer
//    products over all slab rows) and the loss gradient.  The contraction runs
//    over slab rows (K = N*S up to 3e5), so K is split across workgroups; each
//    split writes a partial tile and reduce_splitk sums them in FP64 in a fixed
//    order (deterministic).
#include "common.h"
#include "launch.h"

namespace kp {

template <typename TS> struct TileCfg;
template <> struct TileCfg<bf16> { static constexpr int BM = 128, BN = 128, BK = 32, PAD = 8; };
template <> struct TileCfg<float> { static constexpr int BM = 128, BN = 128, BK = 16, PAD = 4; };
template <> struct TileCfg<double> { static constexpr int BM = 64, BN = 64, BK = 16, PAD = 2; };

typedef uint4 v16;  // one 16-byte vector

template <typename TS>
__device__ __forceinline__ typename Mfma<TS>::frag load_frag(const TS* base, int lane, int ldk, int k0);

template <>
__device__ __forceinline__ bf16x8 load_frag<bf16>(const bf16* base, int lane, int ldk, int k0) {
  return *(const bf16x8*)(base + (lane & 15) * ldk + k0 + (lane >> 4) * 8);
}
template <>
__device__ __forceinline__ float load_frag<float>(const float* base, int lane, int ldk, int k0) {
  return base[(lane & 15) * ldk + k0 + (lane >> 4)];
}
template <>
__device__ __forceinline__ double load_frag<double>(const double* base, int lane, int ldk, int k0) {
  return base[(lane & 15) * ldk + k0 + (lane >> 4)];
}

// XCD-aware tile order: the hardware deals consecutive workgroups round-robin
// to the 8 XCDs; remap so that each XCD receives a contiguous run of logical
// tiles (tiles that share slab rows then share one L2).
__device__ __forceinline__ int xcd_remap(int b, int total) {
  const int per = total / 8, rem = total % 8;
  const int x = b % 8, i = b / 8;
  // XCD x owns logical tiles [x*per + min(x, rem), ...) of length per + (x < rem)
  return x * per + (x < rem ? x : rem) + i;
}

// ---------------------------------------------------------------------------
// C = A * B^T   (A: M x K, B: N x K, K contiguous)
// ---------------------------------------------------------------------------
template <typename TS, bool HILO>
__global__ __launch_bounds__(256) void k_gemm_nt(const TS* __restrict__ A, long lda,
                                                 const TS* __restrict__ B,
                                                 const TS* __restrict__ B2, long ldb, int M, int N,
                                                 int K, typename Acc<TS>::type* __restrict__ out,
                                                 long ldo,
                                                 const typename Acc<TS>::type* __restrict__ bias,
                                                 int S) {
  typedef TileCfg<TS> C;
  typedef Mfma<TS> MF;
  typedef typename Acc<TS>::type TC;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, LDK = BK + C::PAD;
  constexpr int VN = 16 / sizeof(TS);
  constexpr int VPR = BK / VN;
  constexpr int AV = BM * VPR / 256, BV = BN * VPR / 256;
  constexpr int WTM = BM / 2, WTN = BN / 2, TI = WTM / 16, TJ = WTN / 16;
  constexpr int NB = HILO ? 2 : 1;
  __shared__ __align__(16) TS As[2][BM * LDK];
  __shared__ __align__(16) TS Bs[2][NB][BN * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int ntn = gridDim.x, total = gridDim.x * gridDim.y;
  const int t = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, total);
  const int m0 = (t / ntn) * BM, n0 = (t % ntn) * BN;

  v16 ra[AV], rb[NB][BV];
  const v16 z16 = {0u, 0u, 0u, 0u};
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AV; i++) {
      int v = tid + i * 256, r = v / VPR, kv = (v % VPR) * VN;
      int gr = m0 + r, gk = k0 + kv;
      ra[i] = (gr < M && gk < K) ? *(const v16*)(A + (long)gr * lda + gk) : z16;
    }
#pragma unroll
    for (int i = 0; i < BV; i++) {
      int v = tid + i * 256, r = v / VPR, kv = (v % VPR) * VN;
      int gr = n0 + r, gk = k0 + kv;
      bool ok = gr < N && gk < K;
      rb[0][i] = ok ? *(const v16*)(B + (long)gr * ldb + gk) : z16;
      if (HILO) rb[NB - 1][i] = ok ? *(const v16*)(B2 + (long)gr * ldb + gk) : z16;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AV; i++) {
      int v = tid + i * 256, r = v / VPR, kv = (v % VPR) * VN;
      *(v16*)(&As[buf][r * LDK + kv]) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BV; i++) {
      int v = tid + i * 256, r = v / VPR, kv = (v % VPR) * VN;
#pragma unroll
      for (int h = 0; h < NB; h++) *(v16*)(&Bs[buf][h][r * LDK + kv]) = rb[h][i];
    }
  };

  typename MF::acc acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; i++)
#pragma unroll
    for (int j = 0; j < TJ; j++)
#pragma unroll
      for (int e = 0; e < 4; e++) acc[i][j][e] = 0;

  const int nk = (K + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += MF::K) {
      typename MF::frag a[TI], b[NB][TJ];
#pragma unroll
      for (int i = 0; i < TI; i++)
        a[i] = load_frag<TS>(&As[cur][(wm * WTM + i * 16) * LDK], lane, LDK, kk);
#pragma unroll
      for (int h = 0; h < NB; h++)
#pragma unroll
        for (int j = 0; j < TJ; j++)
          b[h][j] = load_frag<TS>(&Bs[cur][h][(wn * WTN + j * 16) * LDK], lane, LDK, kk);
#pragma unroll
      for (int i = 0; i < TI; i++)
#pragma unroll
        for (int j = 0; j < TJ; j++) {
          acc[i][j] = MF::mma(a[i], b[0][j], acc[i][j]);
          if (HILO) acc[i][j] = MF::mma(a[i], b[NB - 1][j], acc[i][j]);
        }
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TI; i++)
#pragma unroll
    for (int j = 0; j < TJ; j++) {
      const int col = n0 + wn * WTN + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int row = m0 + wm * WTM + i * 16 + MF::row(lane, e);
        if (row < M) {
          TC v = (TC)acc[i][j][e];
          if (bias != nullptr && row % S == 0) v += bias[col];
          out[(long)row * ldo + col] = v;
        }
      }
    }
}

hipError_t gemm_nt(Prec p, const void* A, long lda, const void* B, const void* B2, long ldb,
                   int M, int N, int K, void* out, long ldo, const void* bias, int S,
                   hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  switch (p) {
    case P_BF16: {
      dim3 g(kp_cdiv(N, 128), kp_cdiv(M, 128));
      int Kr = (int)kp_roundup(K, 8);
      if (B2)
        k_gemm_nt<bf16, true><<<g, 256, 0, st>>>((const bf16*)A, lda, (const bf16*)B,
                                                 (const bf16*)B2, ldb, M, N, Kr, (float*)out, ldo,
                                                 (const float*)bias, S);
      else
        k_gemm_nt<bf16, false><<<g, 256, 0, st>>>((const bf16*)A, lda, (const bf16*)B, nullptr,
                                                  ldb, M, N, Kr, (float*)out, ldo,
                                                  (const float*)bias, S);
      break;
    }
    case P_F32: {
      dim3 g(kp_cdiv(N, 128), kp_cdiv(M, 128));
      int Kr = (int)kp_roundup(K, 4);
      k_gemm_nt<float, false><<<g, 256, 0, st>>>((const float*)A, lda, (const float*)B, nullptr,
                                                 ldb, M, N, Kr, (float*)out, ldo,
                                                 (const float*)bias, S);
      break;
    }
    case P_F64: {
      dim3 g(kp_cdiv(N, 64), kp_cdiv(M, 64));
      int Kr = (int)kp_roundup(K, 2);
      k_gemm_nt<double, false><<<g, 256, 0, st>>>((const double*)A, lda, (const double*)B,
                                                  nullptr, ldb, M, N, Kr, (double*)out, ldo,
                                                  (const double*)bias, S);
      break;
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// part[s] = sum_{k in split s} w(k) A[k]^T B[k]   (A: K x M, B: K x N, rows)
// ---------------------------------------------------------------------------
template <typename TS, bool WEIGHTED>
__global__ __launch_bounds__(256) void k_gemm_tn(const TS* __restrict__ A, long lda,
                                                 const TS* __restrict__ B, long ldb, int M, int N,
                                                 int K, const double* __restrict__ rw, int S,
                                                 int sym, int ntm, int ntn, int kchunk,
                                                 typename Acc<TS>::type* __restrict__ part) {
  typedef TileCfg<TS> C;
  typedef Mfma<TS> MF;
  typedef typename Acc<TS>::type TC;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, LDK = BK + C::PAD;
  constexpr int VN = 16 / sizeof(TS);
  constexpr int AV = BK * BM / VN / 256, BV = BK * BN / VN / 256;
  constexpr int WTM = BM / 2, WTN = BN / 2, TI = WTM / 16, TJ = WTN / 16;
  __shared__ __align__(16) TS As[2][BM * LDK];
  __shared__ __align__(16) TS Bs[2][BN * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // tile of this workgroup (upper triangle only when sym)
  int ti, tj;
  {
    int t = blockIdx.x;
    if (sym) {
      ti = 0;
      int rowlen = ntm;
      while (t >= rowlen) { t -= rowlen; ti++; rowlen--; }
      tj = ti + t;
    } else {
      ti = t / ntn;
      tj = t % ntn;
    }
  }
  const int m0 = ti * BM, n0 = tj * BN;
  const int split = blockIdx.y;
  const int kbeg = split * kchunk, kend = min(K, kbeg + kchunk);
  const int Mv = (int)kp_roundup(M, VN), Nv = (int)kp_roundup(N, VN);
  TC* out = part + (long)split * M * N;

  TS va[AV][VN], vb[BV][VN];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AV; i++) {
      int v = tid + i * 256, kr = v / (BM / VN), mv = (v % (BM / VN)) * VN;
      int gk = k0 + kr, gm = m0 + mv;
      v16 x = {0u, 0u, 0u, 0u};
      if (gk < kend && gm < Mv) x = *(const v16*)(A + (long)gk * lda + gm);
      const TS* xe = (const TS*)&x;
      if (WEIGHTED) {
        float w = gk < kend ? (float)rw[gk / S] : 0.f;
        if (sizeof(TS) == 8) {
          double wd = gk < kend ? rw[gk / S] : 0.0;
#pragma unroll
          for (int e = 0; e < VN; e++) va[i][e] = cvt<TS>(to_d(xe[e]) * wd);
        } else {
#pragma unroll
          for (int e = 0; e < VN; e++) va[i][e] = from_f<TS>(to_f(xe[e]) * w);
        }
      } else {
#pragma unroll
        for (int e = 0; e < VN; e++) va[i][e] = xe[e];
      }
    }
#pragma unroll
    for (int i = 0; i < BV; i++) {
      int v = tid + i * 256, kr = v / (BN / VN), nv = (v % (BN / VN)) * VN;
      int gk = k0 + kr, gn = n0 + nv;
      v16 x = {0u, 0u, 0u, 0u};
      if (gk < kend && gn < Nv) x = *(const v16*)(B + (long)gk * ldb + gn);
      const TS* xe = (const TS*)&x;
#pragma unroll
      for (int e = 0; e < VN; e++) vb[i][e] = xe[e];
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AV; i++) {
      int v = tid + i * 256, kr = v / (BM / VN), mv = (v % (BM / VN)) * VN;
#pragma unroll
      for (int e = 0; e < VN; e++) As[buf][(mv + e) * LDK + kr] = va[i][e];
    }
#pragma unroll
    for (int i = 0; i < BV; i++) {
      int v = tid + i * 256, kr = v / (BN / VN), nv = (v % (BN / VN)) * VN;
#pragma unroll
      for (int e = 0; e < VN; e++) Bs[buf][(nv + e) * LDK + kr] = vb[i][e];
    }
  };

  typename MF::acc acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; i++)
#pragma unroll
    for (int j = 0; j < TJ; j++)
#pragma unroll
      for (int e = 0; e < 4; e++) acc[i][j][e] = 0;

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kbeg);
    sstore(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += MF::K) {
      typename MF::frag a[TI], b[TJ];
#pragma unroll
      for (int i = 0; i < TI; i++)
        a[i] = load_frag<TS>(&As[cur][(wm * WTM + i * 16) * LDK], lane, LDK, kk);
#pragma unroll
      for (int j = 0; j < TJ; j++)
        b[j] = load_frag<TS>(&Bs[cur][(wn * WTN + j * 16) * LDK], lane, LDK, kk);
#pragma unroll
      for (int i = 0; i < TI; i++)
#pragma unroll
        for (int j = 0; j < TJ; j++) acc[i][j] = MF::mma(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TI; i++)
#pragma unroll
    for (int j = 0; j < TJ; j++) {
      const int col = n0 + wn * WTN + j * 16 + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int row = m0 + wm * WTM + i * 16 + MF::row(lane, e);
        if (row < M) out[(long)row * N + col] = (TC)acc[i][j][e];
      }
    }
}

hipError_t gemm_tn_splitk(Prec p, const void* A, long lda, const void* B, long ldb, int M, int N,
                          int K, const double* rw, int S, bool sym, void* part, int max_splits,
                          int* splits_out, hipStream_t st) {
  const int BT = (p == P_F64) ? 64 : 128;
  const int BK = (p == P_BF16) ? 32 : 16;
  const int ntm = kp_cdiv(M, BT), ntn = kp_cdiv(N, BT);
  const int ntiles = sym ? ntm * (ntm + 1) / 2 : ntm * ntn;
  // enough workgroups to cover the chip a few times, at least 8 k-tiles each
  int splits = kp_cdiv(1024, ntiles);
  int max_by_k = kp_cdiv(K, 8 * BK);
  if (splits > max_by_k) splits = max_by_k;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  int kchunk = (int)kp_roundup(kp_cdiv(K, splits), BK);
  splits = kp_cdiv(K, kchunk);
  if (splits < 1) splits = 1;
  *splits_out = splits;
  dim3 g(ntiles, splits);
  switch (p) {
    case P_BF16:
      if (rw)
        k_gemm_tn<bf16, true><<<g, 256, 0, st>>>((const bf16*)A, lda, (const bf16*)B, ldb, M, N,
                                                 K, rw, S, sym, ntm, ntn, kchunk, (float*)part);
      else
        k_gemm_tn<bf16, false><<<g, 256, 0, st>>>((const bf16*)A, lda, (const bf16*)B, ldb, M, N,
                                                  K, rw, S, sym, ntm, ntn, kchunk, (float*)part);
      break;
    case P_F32:
      if (rw)
        k_gemm_tn<float, true><<<g, 256, 0, st>>>((const float*)A, lda, (const float*)B, ldb, M,
                                                  N, K, rw, S, sym, ntm, ntn, kchunk,
                                                  (float*)part);
      else
        k_gemm_tn<float, false><<<g, 256, 0, st>>>((const float*)A, lda, (const float*)B, ldb, M,
                                                   N, K, rw, S, sym, ntm, ntn, kchunk,
                                                   (float*)part);
      break;
    case P_F64:
      if (rw)
        k_gemm_tn<double, true><<<g, 256, 0, st>>>((const double*)A, lda, (const double*)B, ldb,
                                                   M, N, K, rw, S, sym, ntm, ntn, kchunk,
                                                   (double*)part);
      else
        k_gemm_tn<double, false><<<g, 256, 0, st>>>((const double*)A, lda, (const double*)B, ldb,
                                                    M, N, K, rw, S, sym, ntm, ntn, kchunk,
                                                    (double*)part);
      break;
  }
  return hipGetLastError();
}

template <typename TP>
__global__ void k_reduce_splitk(const TP* __restrict__ part, int splits, int M, int N, int sym,
                                double* __restrict__ out, long so_m, long so_n, double alpha,
                                double c_prev) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M * N) return;
  int m = (int)(idx / N), n = (int)(idx % N);
  if (sym && n < m) return;
  double s = 0.0;
  for (int k = 0; k < splits; k++) s += (double)part[(long)k * M * N + idx];
  double* o = out + m * so_m + n * so_n;
  double v = alpha * s + (c_prev != 0.0 ? c_prev * *o : 0.0);
  *o = v;
  if (sym && n != m) {
    double* o2 = out + n * so_m + m * so_n;
    *o2 = v;   // the lower triangle equals the upper triangle before and after the update
  }
}

hipError_t reduce_splitk(Prec p, const void* part, int splits, int M, int N, bool sym,
                         double* out, long so_m, long so_n, double alpha, double c_prev,
                         hipStream_t st) {
  long tot = (long)M * N;
  int nb = kp_cdiv(tot, 256);
  if (p == P_F64)
    k_reduce_splitk<double><<<nb, 256, 0, st>>>((const double*)part, splits, M, N, sym, out,
                                                so_m, so_n, alpha, c_prev);
  else
    k_reduce_splitk<float><<<nb, 256, 0, st>>>((const float*)part, splits, M, N, sym, out, so_m,
                                               so_n, alpha, c_prev);
  return hipGetLastError();
}

}  // namespace kp
