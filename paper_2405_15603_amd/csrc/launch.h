// Internal launcher interface between the host orchestration (api.cpp) and the
// kernel translation units.  Every launcher enqueues on `st` and returns the
// hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kp {

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_F16 = 3 };

// ---- factor / gradient products (modes of fwdlap.h) -------------------------
// part[s][m*N + n] = sum_{k in split s} w(k) A[k][m] B[k][n] for the tiles the
// kernel covers (sym: only tiles at or above the diagonal).  w(k) = rw[k % rmod]
// when rw != nullptr (one weight per point; slab rows are s-major), else 1;
// the BF16x3 mode reads the FP32 copy rwf of the weights instead.  A and B are
// row-major K x (>= M / N, rounded up to 4) with lda/ldb.  part is double for
// FP64, float otherwise.  The launcher picks the number of splits (<= max_splits).
// wsc: 2 floats of device scratch for the FP16 path's row-weight scaling (needed
// with rw in mode M_F16).
hipError_t gemm_tn_splitk(int mode, const void* A, long lda, const void* B, long ldb, int M, int N,
                          int K, const double* rw, const float* rwf, int rmod, bool sym,
                          void* part, int max_splits, int* splits_out, hipStream_t st,
                          float* wsc = nullptr);
// Grouped factor and gradient products (GroupBlk below): a job holds the
// arguments of one split-K product of the mixed modes (M_BF16X3, M_F16; FP32
// operands, FP32 partial sums), with the split count and grid gemm_tn_splitk
// chooses; the reduction job sums its partials as reduce_splitk does.  The
// FP16 weighted product needs its row scale (row_scale_group) first.
struct TnJob {
  const float* A;
  long lda;
  const float* B;
  long ldb;
  int M, N, K;
  const float* rw;   // FP32 row weights (nullptr: unweighted)
  int rmod, sym, ntm, ntn, kchunk;
  float* part;
  float* wsc;        // FP16: the row-weight scale (2 floats)
  int splits;
};
struct RedJob {
  const float* part;
  int splits, M, N, sym;
  double* out;
  long so_m, so_n;
  double alpha, c_prev;
};
struct GroupBlk;
bool make_tn_job(int mode, const float* A, long lda, const float* B, long ldb, int M, int N, int K,
                 const float* rwf, int rmod, bool sym, float* part, int max_splits, float* wsc,
                 TnJob* j, int* nblk);
RedJob make_red_job(const TnJob& t, double* out, long so_m, long so_n, double alpha,
                    double c_prev, int* nblk);
hipError_t tn_group(int mode, bool weighted, const TnJob* jobs, const GroupBlk* blk, int nblk,
                    hipStream_t st);
hipError_t row_scale_group(const TnJob* jobs, int njobs, hipStream_t st);
hipError_t reduce_group(const RedJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st);

// out[m*so_m + n*so_n] = c_prev*out + alpha * sum_s part[s][m*N+n]  (double out);
// with sym the lower triangle is mirrored from the upper.
hipError_t reduce_splitk(int mode, const void* part, int splits, int M, int N, bool sym,
                         double* out, long so_m, long so_n, double alpha, double c_prev,
                         hipStream_t st);

// ---- elementwise ------------------------------------------------------------
struct LayerDesc {
  int h_in, h_out;
  long off;          // offset of the layer in theta
  long ldk_in;       // row length of the forward weight copy (>= h_in+1)
  long ldk_out;      // row length of the backward weight copy (>= h_out)
  long wrm, wcm;     // element offsets of the two copies in the weight buffer
};
struct NetDesc {
  int L;
  LayerDesc l[8];
};
// Builds the product-layout copies of W~ = theta (+ alpha*dir) for all layers:
// forward copy (h_out x ldk_in, bias in column h_in) and backward copy
// (h_in x ldk_out, W transposed, no bias), plus biases (compute type) and, for
// BF16, the residual low parts.  fwd_only: the forward copy (and biases) only.
hipError_t prep_weights(Prec p, const void* theta, const void* dir, double alpha, NetDesc nd,
                        void* w_hi, void* w_lo, void* bias, long bias_stride, hipStream_t st,
                        int fwd_only = 0);

// Grouped launches: one launch runs the same kernel for many independent
// instances.  Workgroup b runs workgroup blk[b].local of job blk[b].job (tables
// in device memory, built by the host; every job's workgroups are listed once).
struct GroupBlk {
  int job, local;
};
// Grouped line-search launches (FP32 parameters, BF16 slabs and weight copies);
// each job lists nblk workgroups (prep: nblk per layer, L layers).
struct AxpyJob {   // out = theta + alpha * dir over D entries
  const float* theta;
  const float* dir;
  float* out;
  long D;
  int nblk;
};
struct PrepJob {   // the forward BF16 copy of theta (prep_weights with fwd_only)
  const float* theta;
  void* w_hi;
  NetDesc nd;
  int nblk;
};
struct SlabJob {   // the BF16 input slab of n points (unit directions)
  const float* x;
  void* z;
  long ldz;
  int n, d, S, nblk;
};
hipError_t axpy_group(const AxpyJob* jobs, const GroupBlk* blk, int nblk, double alpha,
                      hipStream_t st);
hipError_t prep_group(const PrepJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st);
hipError_t slab_group(const SlabJob* jobs, const GroupBlk* blk, int nblk, hipStream_t st);

// Input slab Z~^(0): S rows per point (value x, unit rows e_i or the directions
// dirs[k*d .. k*d + d) when dirs is given, zero Laplacian row) plus the bias
// column; n points, d inputs, row length ldz.
hipError_t input_slab(Prec p, const void* x, int n, int d, int S, const double* dirs, void* z,
                      long ldz, hipStream_t st);

// Residual, loss partials and the output seed.  pre: last layer output rows
// (compute type, ldp); y: targets (real); r: residual per point (double) and
// rf its FP32 copy (either may be nullptr);
// g: seed rows (storage type, ldg; nullptr = not written); partial: per-block
// sums of r^2 (double, grid size returned by residual_blocks).
int residual_blocks(int npts);
// Terms of an interior residual beyond c_t d_t u + c_lap Lu - y (inactive when
// mask is null): sum_{i: mask[i] != 0} (c_x x_i d_i u + c_g (d_i u)^2) + c_0, with
// x the points (real, row-major npts x d) and d_i u output row 1 + i.
struct ResidualTerms {
  const void* x = nullptr;
  const float* mask = nullptr;
  int d = 0;
  double c_x = 0.0, c_g = 0.0, c_0 = 0.0;
};
hipError_t residual(Prec p, const void* pre, long ldp, const void* y, int npts, int S,
                    int time_row, double c_t, double c_lap, int lap_row, const ResidualTerms& nl,
                    double* r, float* rf, void* g, long ldg, double* partial, hipStream_t st);
// loss[slot] = scale * sum(partial[0..nb)) (+ loss[slot] if accumulate)
hipError_t finalize_loss(const double* partial, int nb, double scale, double* loss, int slot,
                         int accumulate, hipStream_t st);

// Network outputs for the forward-Laplacian entry point: u, grad, lap (real);
// with input directions (dirs, nullable) the gradient is mapped back to the
// coordinate axes.
hipError_t extract_outputs(Prec p, const void* pre, long ldp, int npts, int S, int d, int lap_row,
                           const double* dirs, void* u, void* grad, void* lap, hipStream_t st);
// Output seed rows of a general cotangent (u_bar, grad_bar, lap_bar; real, nullable).
hipError_t seed_rows(Prec p, const void* u_bar, const void* grad_bar, const void* lap_bar,
                     int npts, int S, int d, int lap_row, const double* dirs, void* g, long ldg,
                     hipStream_t st);
// x_bar[n][k] = sum_j W1[j][k] g1[n*S][j]  (value row of the first layer)
hipError_t input_vjp(Prec p, const void* theta, int h_out, int d, const void* g1, long ldg,
                     int npts, int S, void* x_bar, hipStream_t st);

// ---- optimizer --------------------------------------------------------------
// out = theta + alpha * dir (line-search trial parameters)
hipError_t axpy_theta(Prec p, const void* theta, const void* dir, double alpha, void* out, long D,
                      hipStream_t st);
hipError_t ema_fill(double* a, long n, int dim, int identity, hipStream_t st);
// zero a buffer of whole 32-bit words with a kernel (graph-capture safe)
hipError_t zero_fill(void* p, size_t bytes, hipStream_t st);
// dhat = mu*delta + Delta  (real dhat, real delta, double Delta); use_mom = 0 -> dhat = Delta
hipError_t momentum(Prec p, const double* Delta, const void* delta, double mu, const int* step,
                    void* dhat, long D, hipStream_t st);
// alpha* from candidate losses; then theta += alpha*dhat, delta = alpha*dhat;
// writes info and status.  fixed_lr >= 0 -> fixed mode.
hipError_t finish_step(Prec p, const double* losses, int ncand, int kmax, double fixed_lr,
                       double mu, const double* base_loss, void* theta, void* dhat, void* delta,
                       long D, int* status, int* step, void* info, hipStream_t st);

// ---- KFAC* (automatic learning rate and momentum) ---------------------------
// Per-point Jacobian-vector products of the residuals along two directions from
// one layer's stored slabs: jv[dir * ldjv + n] (+)= sum_s g_{n,s}^T D_dir z~_{n,s}
// (dir 0: d0, double; dir 1: d1, the parameter type; both at the layer's offset
// in the theta layout, column-major H x K).  zin: n*S rows of ldz, g: n*S rows of
// ldg (slab type: double for P_F64, float for P_F32).  part: 2 * jvp_tiles(H) *
// n * S slab-type elements of scratch.
int jvp_tiles(int h_out);
hipError_t jvp_layer(Prec p, const void* zin, long ldz, const void* g, long ldg, int n, int S,
                     int K, int H, const double* d0, const void* d1, void* part, double* jv,
                     long ldjv, int accumulate, hipStream_t st);
// The 2 x 2 quadratic model from the products (interior jvi, boundary jvb, two
// rows each of ldi / ldb), Delta, delta_{t-1} (parameter type), the gradient and
// lambda; then delta = alpha Delta + mu delta_{t-1}, theta += delta (skipped when
// the status is set).  Writes alpha and mu into the two doubles after the status
// word and the step summary into info (may be null).
hipError_t kstar_finish(Prec p, const double* jvi, long ldi, int N, const double* jvb, long ldb,
                        int M, const double* Delta, void* delta, const double* grad, long D,
                        double lambda, const double* base_loss, int* status, int* step,
                        void* theta, void* info, hipStream_t st);

// ---- sampler ----------------------------------------------------------------
struct SamplerDesc {
  uint64_t seed_i, seed_b, seed_0;
  int n_i, n_b, n_0, d, face_lo, kind;
  double scale, kappa;
  long step;
};
hipError_t sample(Prec p, SamplerDesc s, void* xi, void* yi, void* xb, void* yb, hipStream_t st);

// ---- FP64 linear algebra for the Kronecker-sum inverse ---------------------
// All problems are padded to n_pad (multiple of 64) square, row-major.
struct EigProblem {
  int n, n_pad;
  const double* f1;   // interior factor (n x n, row-major, EMA state)
  const double* f2;   // boundary factor
  double* M1;         // n_pad^2 work: damped F1, trailing updates
  double* M2;         // n_pad^2 work: damped F2, then scratch
  double* Lb;         // n_pad^2: Cholesky factor L
  double* Li;         // n_pad^2: L^-1
  double* C[2];       // n_pad^2: C[0] whitened F2 rotated by Jacobi, C[1] scratch
  double* P[2];       // n_pad^2: P[0] accumulated rotations V (kept for warm starts),
                      // P[1] the result L^-T V
  double* V;          // (n_pad/64) * 64*64: pair rotations of one round
  int* pflag;         // n_pad/64 + 1 ints: pair is identity this round; last = rotation flag
  double* dmax;       // largest diagonal entry of C (absolute rotation threshold)
  double* Pout;       // n x n result P (row-major)
  double* eout;       // n eigenvalues
  int* status;        // the owning context's status word (nullptr: the call's)
};
// status: the status word of problems without their own; done: 2 ints per
// problem (converged flag, sweeps used); calls: call counter and warm-start flag.
// The problems may belong to several contexts (a batch inverts all of its
// instances' factors in one call).  Jacobi starts from the
// V left in P[0] by the previous call, except on every refresh-th call (and the
// first after the counter is reset).
// The Jacobi sweeps run in up to kEigGroups groups of problems, group k on
// stream st[k] (k = 0: the call's stream, st[0] unused); the other streams fork
// from the call's stream at `fork` and it waits for each at join[k].  Group k
// holds the problems ids[off[k] .. off[k+1]) (ids: device, grouped problem
// indices) and sweeps rounds sized for its largest problem, npmax[k].
// Early stop: with `host` set (eig_host_sync) and the call's stream not being
// captured into a graph, each group's convergence flags are copied to pinned host
// memory after every sweep and read one sweep later; a group whose problems have
// all converged gets no further sweeps.  The launches left out would have returned
// at once (every launch of a converged problem does), so the results equal the
// full schedule's; the call then waits on the host for each sweep but the last.
constexpr int kEigGroups = 4;
struct EigGroups {
  int n = 1;
  int off[kEigGroups + 1] = {};
  int npmax[kEigGroups] = {};
  const int* ids = nullptr;
  hipStream_t st[kEigGroups] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kEigGroups] = {};
  int* host = nullptr;              // pinned: ids (nprob), then 2 x kEigGroups flag copies
  int host_nprob = 0;
  bool host_wait = true;           // early stop allowed (kfac_pinn_set_sweep_wait)
  hipEvent_t swept[kEigGroups][2] = {};
  // With the early stop, a group's sweep (its rounds, the convergence check and
  // the flag copy for one parity) is one captured graph, launched once per sweep:
  // a sweep is ~200 launches, more host time than its GPU time.  Captured on
  // first use on a private stream, for the arguments in sweep_key.
  hipGraphExec_t sweep[kEigGroups][2] = {};
  hipGraph_t sweep_graph[kEigGroups][2] = {};
  hipStream_t cap = nullptr;
  const void* sweep_key[3] = {};
};
// Splits nprob problems into min(ngroups, nprob, kEigGroups) groups of balanced
// work (largest first to the lightest group); fills g.n, g.off, g.npmax and the
// host array ids (nprob ints, to be copied to the device for g.ids).
void eig_groups_plan(const EigProblem* probs, int nprob, int ngroups, int* ids, EigGroups& g);
// Pinned host copies and events of the early stop (ids: the host array of
// eig_groups_plan); eig_host_free releases them.
hipError_t eig_host_sync(EigGroups& g, const int* ids, int nprob);
void eig_host_free(EigGroups& g);
hipError_t kron_eig_batched(const EigProblem* probs_host, int nprob, double lambda,
                            EigProblem* probs_dev, int* status, int* done, int* calls,
                            int refresh, int max_sweeps, EigGroups& g, hipStream_t st);
// Delta = -P_B [(P_B^T V P_A) / (1 + b a^T)] P_A^T for every layer, V = gradient
// (column-major h_out x (h_in+1) inside the theta layout).  Four strided FP64
// products per layer, described once (descriptors in device memory).
struct KronApply {
  int nA, nB;
  long off;                 // layer offset in theta
  const double *PA, *a, *PB, *b;
};
struct G64 {                // C[i*sci + j*scj] = alpha sum_k A(i,k) B(k,j) [/(1 + eb_i ea_j)]
  const double* A;
  long sai, sak;
  const double* B;
  long sbk, sbj;
  double* C;
  long sci, scj;
  int M, N, K;
  double alpha;
  const double* ea;
  const double* eb;
};
// fills h[4*L] (host) for the given buffers; tmp needs L * tmp_stride doubles,
// tmp_stride >= 2 * nA * nB of every layer
void kron_apply_descs(const KronApply* layers, int L, const double* grad, double* delta,
                      double* tmp, long tmp_stride, G64* h, int* mmax, int* nmax);
hipError_t kron_apply_batched(const G64* descs_dev, int L, int mmax, int nmax, hipStream_t st);
// One FP64 product C = alpha A B (+ the optional scaling) with its descriptor as
// the kernel argument.
hipError_t gemm64_one(const G64& g, hipStream_t st);
// Exact Gramian block of one layer and term from its stored slabs (slab type
// P_F64 / P_F32): work (n x p doubles, p = K H) receives the per-point Jacobians
// sum_s z~_{n,s} (x) g_{n,s}, out (p x p doubles) J^T J / n.
hipError_t layer_gramian(Prec p, const void* zin, long ldz, const void* g, long ldg, int n, int S,
                         int K, int H, double* work, double* out, hipStream_t st);
// The same for one layer (layer.off ignored: grad and delta point at the layer's
// block) with its two intermediate products in a static device array of
// 2 * kKronScratchElems doubles and the descriptors as kernel arguments: nothing
// is allocated.  hipErrorInvalidValue when nA * nB > kKronScratchElems.
constexpr long kKronScratchElems = 1L << 20;
hipError_t kron_apply_noalloc(const KronApply& layer, const double* grad, double* delta,
                              hipStream_t st);

}  // namespace kp
