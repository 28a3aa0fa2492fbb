// Elementwise and per-point kernels of the hot path.
//
// Slab layout (all slabs, s-major): row r = s*N + n holds point n's shared
// column s of Z_n (Section 3.2): s = 0 the value, s = 1..d the first
// derivatives, s = S-1 the (masked) Laplacian row.  A boundary slab has S = 1.
// Columns are neurons; layer inputs carry the bias feature in column h
// (1 in the value row, 0 elsewhere, Eq. forward-laplacian-linear-layer-compact)
// and zeros up to the padded row length.
#include "common.h"
#include "launch.h"

namespace kp {

// ---------------------------------------------------------------------------
// Product-layout copies of the augmented weights W~ = [W | b]
// ---------------------------------------------------------------------------
template <typename TP, typename TS>
__device__ __forceinline__ void prep_weights_at(const TP* __restrict__ theta,
                                                const TP* __restrict__ dir, double alpha,
                                                const LayerDesc& ld, int l, TS* __restrict__ whi,
                                                TS* __restrict__ wlo,
                                                typename Acc<TS>::type* __restrict__ bias,
                                                long bias_stride, int fwd_only, long bx, long gx) {
  typedef typename Acc<TS>::type TC;
  const long nf = (long)ld.h_out * ld.ldk_in;    // forward copy elements
  const long nb = fwd_only ? 0 : (long)ld.h_in * ld.ldk_out;   // backward copy elements
  for (long e = bx * blockDim.x + threadIdx.x; e < nf + nb + ld.h_out; e += gx * blockDim.x) {
    long src = -1, dst;
    if (e < nf) {                         // forward: row i (output), column j (input, bias at h_in)
      int i = (int)(e / ld.ldk_in), j = (int)(e % ld.ldk_in);
      dst = ld.wrm + e;
      if (j <= ld.h_in) src = ld.off + (long)j * ld.h_out + i;
    } else if (e < nf + nb) {             // backward: row j (input), column i (output)
      long f = e - nf;
      int j = (int)(f / ld.ldk_out), i = (int)(f % ld.ldk_out);
      dst = ld.wcm + f;
      if (i < ld.h_out) src = ld.off + (long)j * ld.h_out + i;
    } else {                              // bias (compute type)
      int i = (int)(e - nf - nb);
      double w = (double)theta[ld.off + (long)ld.h_in * ld.h_out + i];
      if (dir) w = (double)(TP)((TP)w + (TP)(alpha * (double)dir[ld.off + (long)ld.h_in * ld.h_out + i]));
      if (bias) bias[l * bias_stride + i] = (TC)w;
      continue;
    }
    double w = 0.0;
    if (src >= 0) {
      TP t = theta[src];
      if (dir) t = (TP)(t + (TP)(alpha * (double)dir[src]));
      w = (double)t;
    }
    TS hi = cvt<TS>(w);
    whi[dst] = hi;
    if (wlo) wlo[dst] = cvt<TS>(w - to_d(hi));
  }
}
template <typename TP, typename TS>
__global__ void k_prep_weights(const TP* __restrict__ theta, const TP* __restrict__ dir,
                               double alpha, NetDesc nd, TS* __restrict__ whi,
                               TS* __restrict__ wlo, typename Acc<TS>::type* __restrict__ bias,
                               long bias_stride, int fwd_only) {
  const int l = blockIdx.y;
  if (l >= nd.L) return;
  prep_weights_at<TP, TS>(theta, dir, alpha, nd.l[l], l, whi, wlo, bias, bias_stride, fwd_only,
                          blockIdx.x, gridDim.x);
}

hipError_t prep_weights(Prec p, const void* theta, const void* dir, double alpha, NetDesc nd,
                        void* w_hi, void* w_lo, void* bias, long bias_stride, hipStream_t st,
                        int fwd_only) {
  dim3 g(256, nd.L);
  switch (p) {
    case P_F64:
      k_prep_weights<double, double><<<g, 256, 0, st>>>((const double*)theta, (const double*)dir,
                                                        alpha, nd, (double*)w_hi, nullptr,
                                                        (double*)bias, bias_stride, fwd_only);
      break;
    case P_F32:
      k_prep_weights<float, float><<<g, 256, 0, st>>>((const float*)theta, (const float*)dir,
                                                      alpha, nd, (float*)w_hi, nullptr,
                                                      (float*)bias, bias_stride, fwd_only);
      break;
    case P_BF16:
      k_prep_weights<float, bf16><<<g, 256, 0, st>>>((const float*)theta, (const float*)dir,
                                                     alpha, nd, (bf16*)w_hi, (bf16*)w_lo,
                                                     (float*)bias, bias_stride, fwd_only);
      break;
    case P_F16:
      k_prep_weights<float, f16><<<g, 256, 0, st>>>((const float*)theta, (const float*)dir,
                                                    alpha, nd, (f16*)w_hi, (f16*)w_lo, (float*)bias,
                                                    bias_stride, fwd_only);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Input slab Z~^(0) (Section 3.1: z = x, d_i z = e_i, Lap z = 0; with input
// directions v_k the derivative rows are v_k instead of the unit vectors)
// ---------------------------------------------------------------------------
template <typename TP, typename TS>
__device__ __forceinline__ void input_slab_at(const TP* __restrict__ x, int n, int d, int S,
                                              const double* __restrict__ dirs, TS* __restrict__ z,
                                              long ldz, long bx, long gx) {
  const long R = (long)n * S;
  for (long e = bx * blockDim.x + threadIdx.x; e < R * ldz; e += gx * blockDim.x) {
    long r = e / ldz;
    int j = (int)(e % ldz);
    int s = (int)(r / n), pt = (int)(r % n);
    double v = 0.0;
    if (s == 0) v = j < d ? (double)x[(long)pt * d + j] : (j == d ? 1.0 : 0.0);
    else if (S > 1 && s < S - 1)
      v = dirs ? (j < d ? dirs[(long)(s - 1) * d + j] : 0.0) : ((j == s - 1) ? 1.0 : 0.0);
    z[e] = cvt<TS>(v);
  }
}
template <typename TP, typename TS>
__global__ void k_input_slab(const TP* __restrict__ x, int n, int d, int S,
                             const double* __restrict__ dirs, TS* __restrict__ z, long ldz) {
  input_slab_at<TP, TS>(x, n, d, S, dirs, z, ldz, blockIdx.x, gridDim.x);
}

hipError_t input_slab(Prec p, const void* x, int n, int d, int S, const double* dirs, void* z,
                      long ldz, hipStream_t st) {
  long tot = (long)n * S * ldz;
  int nb = (int)((tot + 255) / 256);
  if (nb > 65536) nb = 65536;
  if (nb < 1) nb = 1;
  switch (p) {
    case P_F64:
      k_input_slab<double, double><<<nb, 256, 0, st>>>((const double*)x, n, d, S, dirs, (double*)z, ldz);
      break;
    case P_F32:
      k_input_slab<float, float><<<nb, 256, 0, st>>>((const float*)x, n, d, S, dirs, (float*)z, ldz);
      break;
    case P_BF16:
      k_input_slab<float, bf16><<<nb, 256, 0, st>>>((const float*)x, n, d, S, dirs, (bf16*)z, ldz);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Residual (Eq. pinn-loss), loss partials and the output seed d r / d U
// ---------------------------------------------------------------------------
int residual_blocks(int npts) { return npts > 0 ? (npts + 255) / 256 : 1; }

// Interior residuals with first-order terms (Section 3.3: a residual that depends
// on the derivatives non-linearly, e.g. the logarithmic Fokker-Planck equation of
// Section 4):  r += sum_{i in mask} (c_x x_i d_i u + c_g (d_i u)^2) + c_0, whose
// seed on derivative row i is c_x x_i + 2 c_g d_i u (point-dependent).
template <typename TC, typename TP, typename TS>
__global__ __launch_bounds__(256) void k_residual(const TC* __restrict__ pre, long ldp,
                                                  const TP* __restrict__ y, int npts, int S,
                                                  int time_row, double c_t, double c_lap,
                                                  int lap_row, ResidualTerms nl,
                                                  double* __restrict__ r,
                                                  float* __restrict__ rf, TS* __restrict__ g,
                                                  long ldg,
                                                  double* __restrict__ partial) {
  __shared__ double red[4];
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const bool extra = lap_row >= 0 && nl.mask != nullptr;
  const TP* xp = (const TP*)nl.x;
  double sq = 0.0;
  if (n < npts) {
    double v;
    if (lap_row >= 0 || time_row >= 0) {
      v = -(double)y[n];
      if (lap_row >= 0) v += c_lap * (double)pre[((long)lap_row * npts + n) * ldp];
      if (time_row >= 0) v += c_t * (double)pre[((long)time_row * npts + n) * ldp];
      if (extra) {
        v += nl.c_0;
        for (int i = 0; i < nl.d; i++) {
          if (nl.mask[i] == 0.0f) continue;
          const double du = (double)pre[((long)(1 + i) * npts + n) * ldp];
          v += (nl.c_x * (double)xp[(long)n * nl.d + i] + nl.c_g * du) * du;
        }
      }
    } else {
      v = (double)pre[(long)n * ldp] - (double)y[n];   // boundary: r = u - g
    }
    if (r) r[n] = v;
    if (rf) rf[n] = (float)v;
    sq = v * v;
    if (g) {
      for (int s = 0; s < S; s++) {
        double sv = 0.0;
        if (lap_row < 0 && time_row < 0) sv = (s == 0) ? 1.0 : 0.0;
        else {
          if (s == lap_row) sv += c_lap;
          if (s == time_row) sv += c_t;
          if (extra && s >= 1 && s <= nl.d && nl.mask[s - 1] != 0.0f) {
            const double du = (double)pre[((long)s * npts + n) * ldp];
            sv += nl.c_x * (double)xp[(long)n * nl.d + s - 1] + 2.0 * nl.c_g * du;
          }
        }
        const long row = (long)s * npts + n;
        g[row * ldg] = cvt<TS>(sv);
        for (int c = 1; c < ldg; c++) g[row * ldg + c] = cvt<TS>(0.0);
      }
    }
  }
  sq = warp_sum(sq);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

hipError_t residual(Prec p, const void* pre, long ldp, const void* y, int npts, int S,
                    int time_row, double c_t, double c_lap, int lap_row, const ResidualTerms& nl,
                    double* r, float* rf, void* g, long ldg, double* partial, hipStream_t st) {
  int nb = residual_blocks(npts);
  switch (p) {
    case P_F64:
      k_residual<double, double, double><<<nb, 256, 0, st>>>(
          (const double*)pre, ldp, (const double*)y, npts, S, time_row, c_t, c_lap, lap_row, nl, r, rf,
          (double*)g, ldg, partial);
      break;
    case P_F32:
      k_residual<float, float, float><<<nb, 256, 0, st>>>((const float*)pre, ldp,
                                                          (const float*)y, npts, S, time_row, c_t,
                                                          c_lap, lap_row, nl, r, rf, (float*)g, ldg,
                                                          partial);
      break;
    case P_BF16:
      k_residual<float, float, bf16><<<nb, 256, 0, st>>>((const float*)pre, ldp, (const float*)y,
                                                         npts, S, time_row, c_t, c_lap, lap_row,
                                                         nl, r, rf, (bf16*)g, ldg, partial);
      break;
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_finalize_loss(const double* __restrict__ partial, int nb,
                                                       double scale, double* loss, int slot,
                                                       int accumulate) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += partial[i];
  s = warp_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = scale * (red[0] + red[1] + red[2] + red[3]);
    loss[slot] = accumulate ? loss[slot] + v : v;
  }
}

hipError_t finalize_loss(const double* partial, int nb, double scale, double* loss, int slot,
                         int accumulate, hipStream_t st) {
  k_finalize_loss<<<1, 256, 0, st>>>(partial, nb, scale, loss, slot, accumulate);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward-Laplacian outputs and general seeds (autograd entry points)
// ---------------------------------------------------------------------------
// With input directions v_k (rows 1..d hold the derivatives along v_k, V
// orthogonal) the gradient is grad_i = sum_k V[i][k] d_k u, dirs[k*d + i] = V[i][k].
template <typename TC, typename TP>
__global__ void k_extract(const TC* __restrict__ pre, long ldp, int npts, int S, int d,
                          int lap_row, const double* __restrict__ dirs, TP* u, TP* grad, TP* lap) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= npts) return;
  if (u) u[n] = (TP)pre[(long)n * ldp];
  if (grad && dirs)
    for (int i = 0; i < d; i++) {
      double g = 0.0;
      for (int k = 0; k < d; k++)
        g += dirs[(long)k * d + i] * (double)pre[((long)(1 + k) * npts + n) * ldp];
      grad[(long)n * d + i] = (TP)g;
    }
  else if (grad)
    for (int i = 0; i < d; i++) grad[(long)n * d + i] = (TP)pre[((long)(1 + i) * npts + n) * ldp];
  if (lap) lap[n] = lap_row >= 0 ? (TP)pre[((long)lap_row * npts + n) * ldp] : (TP)0;
}

hipError_t extract_outputs(Prec p, const void* pre, long ldp, int npts, int S, int d, int lap_row,
                           const double* dirs, void* u, void* grad, void* lap, hipStream_t st) {
  int nb = (npts + 255) / 256;
  if (nb < 1) return hipSuccess;
  if (p == P_F64)
    k_extract<double, double><<<nb, 256, 0, st>>>((const double*)pre, ldp, npts, S, d, lap_row,
                                                  dirs, (double*)u, (double*)grad, (double*)lap);
  else
    k_extract<float, float><<<nb, 256, 0, st>>>((const float*)pre, ldp, npts, S, d, lap_row,
                                                dirs, (float*)u, (float*)grad, (float*)lap);
  return hipGetLastError();
}

// The cotangent of grad u enters row k as sum_i V[i][k] grad_bar_i with input
// directions (the transpose of k_extract's map).
template <typename TP, typename TS>
__global__ void k_seed(const TP* __restrict__ ub, const TP* __restrict__ gb,
                       const TP* __restrict__ lb, int npts, int S, int d, int lap_row,
                       const double* __restrict__ dirs, TS* g, long ldg) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= npts) return;
  for (int s = 0; s < S; s++) {
    double v = 0.0;
    if (s == 0) v = ub ? (double)ub[n] : 0.0;
    else if (s == lap_row) v = lb ? (double)lb[n] : 0.0;
    else if (s <= d && gb && dirs) {
      for (int i = 0; i < d; i++) v += dirs[(long)(s - 1) * d + i] * (double)gb[(long)n * d + i];
    } else if (s <= d) {
      v = gb ? (double)gb[(long)n * d + s - 1] : 0.0;
    }
    const long row = (long)s * npts + n;
    g[row * ldg] = cvt<TS>(v);
    for (int c = 1; c < ldg; c++) g[row * ldg + c] = cvt<TS>(0.0);
  }
}

hipError_t seed_rows(Prec p, const void* u_bar, const void* grad_bar, const void* lap_bar,
                     int npts, int S, int d, int lap_row, const double* dirs, void* g, long ldg,
                     hipStream_t st) {
  int nb = (npts + 255) / 256;
  if (nb < 1) return hipSuccess;
  switch (p) {
    case P_F64:
      k_seed<double, double><<<nb, 256, 0, st>>>((const double*)u_bar, (const double*)grad_bar,
                                                 (const double*)lap_bar, npts, S, d, lap_row,
                                                 dirs, (double*)g, ldg);
      break;
    case P_F32:
      k_seed<float, float><<<nb, 256, 0, st>>>((const float*)u_bar, (const float*)grad_bar,
                                               (const float*)lap_bar, npts, S, d, lap_row,
                                               dirs, (float*)g, ldg);
      break;
    case P_BF16:
      k_seed<float, bf16><<<nb, 256, 0, st>>>((const float*)u_bar, (const float*)grad_bar,
                                              (const float*)lap_bar, npts, S, d, lap_row,
                                              dirs, (bf16*)g, ldg);
      break;
  }
  return hipGetLastError();
}

template <typename TP, typename TS>
__global__ void k_input_vjp(const TP* __restrict__ theta, int h_out, int d,
                            const TS* __restrict__ g1, long ldg, int npts, int S, TP* xb) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)npts * d) return;
  const int n = (int)(e / d), k = (int)(e % d);
  double s = 0.0;
  const TS* gr = g1 + (long)n * ldg;   // value row s = 0 of point n
  for (int j = 0; j < h_out; j++) s += (double)theta[(long)k * h_out + j] * to_d(gr[j]);
  xb[e] = (TP)s;
}

hipError_t input_vjp(Prec p, const void* theta, int h_out, int d, const void* g1, long ldg,
                     int npts, int S, void* x_bar, hipStream_t st) {
  long tot = (long)npts * d;
  int nb = (int)((tot + 255) / 256);
  if (nb < 1) return hipSuccess;
  switch (p) {
    case P_F64:
      k_input_vjp<double, double><<<nb, 256, 0, st>>>((const double*)theta, h_out, d,
                                                      (const double*)g1, ldg, npts, S,
                                                      (double*)x_bar);
      break;
    case P_F32:
      k_input_vjp<float, float><<<nb, 256, 0, st>>>((const float*)theta, h_out, d,
                                                    (const float*)g1, ldg, npts, S,
                                                    (float*)x_bar);
      break;
    case P_BF16:
      k_input_vjp<float, bf16><<<nb, 256, 0, st>>>((const float*)theta, h_out, d, (const bf16*)g1,
                                                   ldg, npts, S, (float*)x_bar);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Optimizer state (Section 3.4; Algorithm 1 steps 0, 4 and 5)
// ---------------------------------------------------------------------------
__global__ void k_ema_fill(double* a, long n, int dim, int identity) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  a[e] = (identity && (e / dim) == (e % dim)) ? 1.0 : 0.0;
}

// Zero `words` 32-bit words (a kernel, not a memset node, so that captured
// graphs replay it reliably).
__global__ void k_zero_words(uint32_t* __restrict__ p, long words) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t zero_fill(void* p, size_t bytes, hipStream_t st) {
  const long words = (long)(bytes / 4);
  if (words <= 0) return hipSuccess;
  int nb = (int)((words + 255) / 256);
  if (nb > 4096) nb = 4096;
  k_zero_words<<<nb, 256, 0, st>>>((uint32_t*)p, words);
  return hipGetLastError();
}

hipError_t ema_fill(double* a, long n, int dim, int identity, hipStream_t st) {
  k_ema_fill<<<(int)((n + 255) / 256), 256, 0, st>>>(a, n, dim, identity);
  return hipGetLastError();
}

template <typename TP>
__global__ void k_momentum(const double* __restrict__ Delta, const TP* __restrict__ delta,
                           double mu, const int* __restrict__ step, TP* __restrict__ dhat,
                           long D) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D) return;
  const bool mom = *step > 0;
  double v = Delta[e] + (mom ? mu * (double)delta[e] : 0.0);
  dhat[e] = (TP)v;
}

hipError_t momentum(Prec p, const double* Delta, const void* delta, double mu, const int* step,
                    void* dhat, long D, hipStream_t st) {
  int nb = (int)((D + 255) / 256);
  if (p == P_F64)
    k_momentum<double><<<nb, 256, 0, st>>>(Delta, (const double*)delta, mu, step, (double*)dhat, D);
  else
    k_momentum<float><<<nb, 256, 0, st>>>(Delta, (const float*)delta, mu, step, (float*)dhat, D);
  return hipGetLastError();
}

template <typename TP>
__global__ void k_axpy_theta(const TP* __restrict__ theta, const TP* __restrict__ dir, double alpha,
                             TP* __restrict__ out, long D) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D) return;
  out[e] = theta[e] + (TP)(alpha * (double)dir[e]);
}

hipError_t axpy_theta(Prec p, const void* theta, const void* dir, double alpha, void* out, long D,
                      hipStream_t st) {
  int nb = (int)((D + 255) / 256);
  if (p == P_F64)
    k_axpy_theta<double><<<nb, 256, 0, st>>>((const double*)theta, (const double*)dir, alpha,
                                             (double*)out, D);
  else
    k_axpy_theta<float><<<nb, 256, 0, st>>>((const float*)theta, (const float*)dir, alpha,
                                            (float*)out, D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Grouped line-search launches (see GroupBlk): the candidate parameters, their
// BF16 forward copy and both input slabs of many instances, one launch each.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T ld_uniform(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(4))) T*)p;
#else
  return *p;   // the host pass only parses device code
#endif
}

__global__ __launch_bounds__(256) void k_axpy_group(const AxpyJob* __restrict__ jobs,
                                                    const GroupBlk* __restrict__ blk,
                                                    double alpha) {
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const AxpyJob j = ld_uniform(jobs + g.job);
  for (long e = (long)g.local * blockDim.x + threadIdx.x; e < j.D; e += (long)j.nblk * blockDim.x)
    j.out[e] = j.theta[e] + (float)(alpha * (double)j.dir[e]);
}

__global__ __launch_bounds__(256) void k_prep_group(const PrepJob* __restrict__ jobs,
                                                    const GroupBlk* __restrict__ blk) {
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const PrepJob* jp = jobs + g.job;
  const int nblk = ld_uniform(&jp->nblk);
  const int l = g.local / nblk;   // nblk workgroups per layer
  // only this layer's descriptor (a whole NetDesc indexed by l would live in scratch)
  const LayerDesc ld = ld_uniform(&jp->nd.l[l]);
  prep_weights_at<float, bf16>(ld_uniform(&jp->theta), nullptr, 0.0, ld, l,
                               (bf16*)ld_uniform(&jp->w_hi), nullptr, nullptr, 0, 1,
                               g.local - l * nblk, nblk);
}

__global__ __launch_bounds__(256) void k_slab_group(const SlabJob* __restrict__ jobs,
                                                    const GroupBlk* __restrict__ blk) {
  const GroupBlk g = ld_uniform(blk + blockIdx.x);
  const SlabJob j = ld_uniform(jobs + g.job);
  input_slab_at<float, bf16>(j.x, j.n, j.d, j.S, nullptr, (bf16*)j.z, j.ldz, g.local, j.nblk);
}

hipError_t axpy_group(const AxpyJob* jobs, const GroupBlk* blk, int nblk, double alpha,
                      hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  k_axpy_group<<<nblk, 256, 0, st>>>(jobs, blk, alpha);
  return hipGetLastError();
}
hipError_t prep_group(const PrepJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  k_prep_group<<<nblk, 256, 0, st>>>(jobs, blk);
  return hipGetLastError();
}
hipError_t slab_group(const SlabJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st) {
  if (nblk <= 0) return hipSuccess;
  k_slab_group<<<nblk, 256, 0, st>>>(jobs, blk);
  return hipGetLastError();
}

struct StepInfoDev {
  double loss_interior, loss_boundary, lr_chosen, loss_after;
  int status, step;
  double momentum_chosen;   // coefficient of delta_{t-1} in the applied update
};

// alpha* = first strict minimum over candidates ordered from the largest step
// (ties go to the larger alpha); non-finite losses are skipped.
__global__ void k_select(const double* __restrict__ losses, int ncand, int kmax, double fixed_lr,
                         double mu, const double* __restrict__ base, int* status, int* step,
                         double* alpha, StepInfoDev* info) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, after = __builtin_nan("");
  int st = *status;
  // a non-finite loss at theta_t (non-finite points, targets or parameters) is the
  // cause of whatever else failed downstream of it
  if (!isfinite(base[0]) || !isfinite(base[1])) st = 5;
  if (st == 0) {
    if (fixed_lr >= 0.0) {
      a = fixed_lr;
    } else {
      int best = -1;
      double bv = 0.0;
      for (int c = 0; c < ncand; c++) {
        double v = losses[c];
        if (isfinite(v) && (best < 0 || v < bv)) { best = c; bv = v; }
      }
      if (best < 0) st = 5;
      else { a = ldexp(1.0, kmax - best); after = bv; }
    }
  }
  if (st != 0) a = 0.0;
  // delta_t = alpha (mu delta_{t-1} + Delta) carries alpha mu of delta_{t-1}
  // (none at the first step, where delta_{-1} = 0)
  const double mom = (st == 0 && *step > 0) ? a * mu : 0.0;
  *status = st;
  *alpha = a;
  if (st == 0) *step += 1;
  if (info) {
    info->loss_interior = base[0];
    info->loss_boundary = base[1];
    info->lr_chosen = a;
    info->loss_after = after;
    info->status = st;
    info->step = *step;
    info->momentum_chosen = mom;
  }
}

template <typename TP>
__global__ void k_apply_update(const int* __restrict__ status, const double* __restrict__ alpha,
                               TP* __restrict__ theta, const TP* __restrict__ dhat,
                               TP* __restrict__ delta, long D) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= D || *status != 0) return;
  const TP d = (TP)(*alpha * (double)dhat[e]);
  delta[e] = d;
  theta[e] = theta[e] + d;
}

hipError_t finish_step(Prec p, const double* losses, int ncand, int kmax, double fixed_lr,
                       double mu, const double* base_loss, void* theta, void* dhat, void* delta,
                       long D, int* status, int* step, void* info, hipStream_t st) {
  double* alpha = (double*)(status + 4);   // scalar slot next to the status word
  k_select<<<1, 64, 0, st>>>(losses, ncand, kmax, fixed_lr, mu, base_loss, status, step, alpha,
                             (StepInfoDev*)info);
  int nb = (int)((D + 255) / 256);
  if (p == P_F64)
    k_apply_update<double><<<nb, 256, 0, st>>>(status, alpha, (double*)theta,
                                               (const double*)dhat, (double*)delta, D);
  else
    k_apply_update<float><<<nb, 256, 0, st>>>(status, alpha, (float*)theta, (const float*)dhat,
                                              (float*)delta, D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sampler: SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sm64_uniform(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-53;
}

// Targets of the manufactured solutions, from the running sums of one point:
// ssum = sum sin(pi x_i) over all coordinates, hsum = the same over i >= 1.
__device__ __forceinline__ double target_f(double x0, double x1, double ssum, int kind,
                                          double scale) {
  const double pi = 3.14159265358979323846;
  if (kind == 1) return 2.0 * pi * pi * sin(pi * x0) * sin(pi * x1);
  if (kind == 2) return 0.0;
  return scale * pi * pi * ssum;
}
__device__ __forceinline__ double target_g(double x0, double ssum, double hsum, int kind,
                                          double scale, double kappa) {
  const double pi = 3.14159265358979323846;
  if (kind == 1) return 0.0;
  if (kind == 2) return exp(-kappa * pi * pi * x0) * hsum;
  return scale * ssum;
}

template <typename TP>
__global__ void k_sample(SamplerDesc s, TP* xi, TP* yi, TP* xb, TP* yb) {
  const double pi = 3.14159265358979323846;
  const int d = s.d;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  double x0 = 0.0, x1 = 0.0, ssum = 0.0, hsum = 0.0;
  if (n < s.n_i) {
    const uint64_t base = (uint64_t)s.step * s.n_i * d + (uint64_t)n * d;
    for (int j = 0; j < d; j++) {
      const double v = sm64_uniform(s.seed_i, base + j);
      xi[(long)n * d + j] = (TP)v;
      if (j == 0) x0 = v;
      if (j == 1) x1 = v;
      const double sv = sin(pi * v);
      ssum += sv;
      if (j >= 1) hsum += sv;
    }
    yi[n] = (TP)target_f(x0, x1, ssum, s.kind, s.scale);
  } else if (n < s.n_i + s.n_0) {      // initial points: x_0 = 0
    const int m = n - s.n_i;
    const uint64_t base = (uint64_t)s.step * s.n_0 * d + (uint64_t)m * d;
    for (int j = 0; j < d; j++) {
      const double v = j == 0 ? 0.0 : sm64_uniform(s.seed_0, base + j);
      xb[(long)m * d + j] = (TP)v;
      const double sv = sin(pi * v);
      ssum += sv;
      if (j >= 1) hsum += sv;
    }
    yb[m] = (TP)target_g(0.0, ssum, hsum, s.kind, s.scale, s.kappa);
  } else if (n < s.n_i + s.n_0 + s.n_b) {
    const int m = n - s.n_i - s.n_0;
    const uint64_t base = (uint64_t)s.step * s.n_b * (d + 1) + (uint64_t)m * (d + 1);
    const int nf = 2 * (d - s.face_lo);
    int f = (int)floor(sm64_uniform(s.seed_b, base) * nf);
    if (f > nf - 1) f = nf - 1;
    const int fc = s.face_lo + f / 2;
    const int row = s.n_0 + m;
    for (int j = 0; j < d; j++) {
      const double v = j == fc ? (double)(f % 2) : sm64_uniform(s.seed_b, base + 1 + j);
      xb[(long)row * d + j] = (TP)v;
      if (j == 0) x0 = v;
      const double sv = sin(pi * v);
      ssum += sv;
      if (j >= 1) hsum += sv;
    }
    yb[row] = (TP)target_g(x0, ssum, hsum, s.kind, s.scale, s.kappa);
  }
}

hipError_t sample(Prec p, SamplerDesc s, void* xi, void* yi, void* xb, void* yb, hipStream_t st) {
  int tot = s.n_i + s.n_0 + s.n_b;
  int nb = (tot + 127) / 128;
  if (nb < 1) return hipSuccess;
  if (p == P_F64)
    k_sample<double><<<nb, 128, 0, st>>>(s, (double*)xi, (double*)yi, (double*)xb, (double*)yb);
  else
    k_sample<float><<<nb, 128, 0, st>>>(s, (float*)xi, (float*)yi, (float*)xb, (float*)yb);
  return hipGetLastError();
}

}  // namespace kp
