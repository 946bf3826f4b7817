// Vector kernels of the outer Krylov iteration: deterministic batched dot
// products (fixed two-stage tree), the fused CG updates with per-right-hand-
// side masks, precision conversion and fills.  Vectors are [nrhs][n] with a
// per-RHS stride; scalars are device arrays of nrhs doubles.
#include <hip/hip_runtime.h>

#include "dgmg_blas.h"

namespace dgmg {
namespace {

constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

// partial[r][blk] = sum over the block's grid-stride share of a_r . b_r
// (and, if c != nullptr, partial2 = c_r . d_r); vector r of a starts at
// r * sa, of b at r * sb (sb = 0: one b against every a_r).  b and c may be
// FP32 vectors, read as the FP64 values they hold exactly.
template <typename TB>
__global__ void __launch_bounds__(kRedThreads)
k_dot2(const double* __restrict__ a, const TB* __restrict__ b, const TB* __restrict__ c,
       const double* __restrict__ d, long long n, long long sa, long long sb,
       double* __restrict__ partial, double* __restrict__ partial2) {
  __shared__ double sh[kRedThreads];
  const long long off = (long long)blockIdx.y * sa;
  const long long offb = (long long)blockIdx.y * sb;
  double s1 = 0.0, s2 = 0.0;
  const long long stride = (long long)gridDim.x * kRedThreads;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
    s1 += a[off + i] * (double)b[offb + i];
    if (c) s2 += (double)c[off + i] * d[off + i];
  }
  const double r1 = block_sum(s1, sh);
  if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = r1;
  if (c) {
    __syncthreads();
    const double r2 = block_sum(s2, sh);
    if (threadIdx.x == 0) partial2[blockIdx.y * gridDim.x + blockIdx.x] = r2;
  }
}

// sum_blk partial[blk] over nblk first-stage partial sums in a fixed order
// (every thread of the block gets the result): the second stage of every
// reduction, so a sum formed here equals the one k_finalize writes, bit for
// bit, in whichever block or kernel it is formed
__device__ __forceinline__ double sum_partials(const double* __restrict__ partial, int nblk,
                                               double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += kRedThreads) s += partial[i];
  return block_sum(s, sh);
}

// out[r] = sum_blk partial[r][blk] in a fixed order
__global__ void __launch_bounds__(kRedThreads)
k_finalize(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  const double r = sum_partials(partial + blockIdx.x * nblk, nblk, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

// Coefficient gradient of the differentiable solve from the first-stage
// partial sums of lambda_r . (A_1 u_r): out[r] = -(that sum), summed in the
// order of k_finalize; then (block 0 of a second launch) out[nrhs] = the sum of
// out[0..nrhs) in index order, the gradient with respect to one coefficient
// shared by every right-hand side.
__global__ void __launch_bounds__(kRedThreads)
k_neg_finalize(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  const double r = sum_partials(partial + blockIdx.x * nblk, nblk, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = -r;
}
__global__ void k_sum_rhs(double* __restrict__ out, int nrhs) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int r = 0; r < nrhs; ++r) s += out[r];
  out[nrhs] = s;
}

// x += alpha p, r -= alpha q with alpha = rz/pq for active right-hand sides;
// partial sums of |r|^2.  p^T q comes as the nblk first-stage partial sums of
// the preceding dot product (pq_part); every block finishes that sum itself
// (same value in every block) instead of waiting for another launch, and
// block 0 stores it and alpha.
__global__ void __launch_bounds__(kRedThreads)
k_update_xr(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
            const double* __restrict__ q, const double* __restrict__ rz,
            const double* __restrict__ pq_part, int nblk, double* __restrict__ pq_out,
            const int* __restrict__ active, long long n, double* __restrict__ alpha_out,
            double* __restrict__ partial, float* __restrict__ r32) {
  __shared__ double sh[kRedThreads];
  const int rhs = blockIdx.y;
  const long long off = (long long)rhs * n;
  const bool act = active[rhs] != 0;
  const double pq = sum_partials(pq_part + rhs * nblk, nblk, sh);
  __syncthreads();
  const double alpha = act ? rz[rhs] / pq : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    alpha_out[rhs] = alpha;
    pq_out[rhs] = pq;
  }
  double s = 0.0;
  const long long stride = (long long)gridDim.x * kRedThreads;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
    double ri = r[off + i];
    if (act) {
      x[off + i] += alpha * p[off + i];
      ri -= alpha * q[off + i];
      r[off + i] = ri;
      if (r32) r32[off + i] = (float)ri;  // right-hand side of an FP32 V-cycle
    }
    s += ri * ri;
  }
  const double red = block_sum(s, sh);
  if (threadIdx.x == 0) partial[rhs * gridDim.x + blockIdx.x] = red;
}

// Convergence check after the CG update, one block per right-hand side:
// rr = |r|^2 from the update's partial sums; for an active right-hand side
// rel = sqrt(rr) / nb, which stays active while rel > rtol.  The record
// rec[4 rhs ..] = (rr, p^T q, rel, active) goes to host-visible memory, the
// mask to `active` for the kernels of the next iteration.
__global__ void __launch_bounds__(kRedThreads)
k_cg_check(const double* __restrict__ rr_part, int nblk, double* __restrict__ rr_out,
           const double* __restrict__ pq, const double* __restrict__ nb, double rtol,
           int* __restrict__ active, double* __restrict__ rec) {
  __shared__ double sh[kRedThreads];
  const int rhs = blockIdx.x;
  const double r2 = sum_partials(rr_part + rhs * nblk, nblk, sh);
  if (threadIdx.x == 0) {
    rr_out[rhs] = r2;
    const bool act = active[rhs] != 0;
    const double rel = sqrt(r2) / nb[rhs];
    const int still = (act && rel > rtol) ? 1 : 0;
    active[rhs] = still;
    rec[4 * rhs + 0] = r2;
    rec[4 * rhs + 1] = pq[rhs];
    rec[4 * rhs + 2] = rel;
    rec[4 * rhs + 3] = (double)still;
  }
}

// p = z + beta p for active right-hand sides; beta = rz_new/rz_old (standard)
// or -alpha zq / rz_old (flexible: z^T (r_new - r_old) / rz_old).  rz_new
// (and zq) come as the nblk partial sums of the preceding dot product; every
// block finishes them itself, block 0 stores them.  z may be the FP32 output
// of the V-cycle, read as the FP64 values it holds exactly.
template <typename TZ>
__global__ void __launch_bounds__(kRedThreads)
k_update_p(double* __restrict__ p, const TZ* __restrict__ z, const double* __restrict__ rz_part,
           const double* __restrict__ zq_part, int nblk, double* __restrict__ rz_new_out,
           double* __restrict__ zq_out, const double* __restrict__ rz_old,
           const double* __restrict__ alpha, const int* __restrict__ active, int flexible,
           long long n) {
  __shared__ double sh[kRedThreads];
  const int rhs = blockIdx.y;
  if (!active[rhs]) return;
  const long long off = (long long)rhs * n;
  const double rz_new = sum_partials(rz_part + rhs * nblk, nblk, sh);
  double zq = 0.0;
  if (flexible) {
    __syncthreads();
    zq = sum_partials(zq_part + rhs * nblk, nblk, sh);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    rz_new_out[rhs] = rz_new;
    if (flexible) zq_out[rhs] = zq;
  }
  const double beta = flexible ? (-alpha[rhs] * zq / rz_old[rhs]) : (rz_new / rz_old[rhs]);
  const long long stride = (long long)gridDim.x * kRedThreads;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride)
    p[off + i] = (double)z[off + i] + beta * p[off + i];
}

template <typename S, typename T>
__global__ void __launch_bounds__(kRedThreads)
k_convert(const S* __restrict__ a, T* __restrict__ b, long long n) {
  const long long stride = (long long)gridDim.x * kRedThreads;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride)
    b[i] = (T)a[i];
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_fill(T* __restrict__ a, T v, long long n) {
  const long long stride = (long long)gridDim.x * kRedThreads;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) a[i] = v;
}

// w += sgn * sum_{i < m} coef[i] V_i  (V: m vectors at stride n)
__global__ void __launch_bounds__(kRedThreads)
k_multi_axpy(double* __restrict__ w, const double* __restrict__ V, const double* __restrict__ coef,
             int m, double sgn, long long n) {
  const long long stride = (long long)gridDim.x * kRedThreads;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += coef[j] * V[(long long)j * n + i];
    w[i] += sgn * s;
  }
}

// v = w / sqrt(nn[0]) (nn > 0 is checked by the host before the basis is used)
__global__ void __launch_bounds__(kRedThreads)
k_normalise(double* __restrict__ v, double* __restrict__ v2, const double* __restrict__ w,
            const double* __restrict__ nn, long long n) {
  const double inv = 1.0 / sqrt(nn[0]);
  const long long stride = (long long)gridDim.x * kRedThreads;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
    const double y = w[i] * inv;
    v[i] = y;
    if (v2) v2[i] = y;
  }
}

// y = a - b  (residual r = b - A x)
__global__ void __launch_bounds__(kRedThreads)
k_sub(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y,
      long long n) {
  const long long stride = (long long)gridDim.x * kRedThreads;
  for (long long i = (long long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride)
    y[i] = a[i] - b[i];
}

int grid_for(long long n) {
  long long g = (n + kRedThreads * 4 - 1) / (kRedThreads * 4);
  if (g < 1) g = 1;
  if (g > kRedBlocks) g = kRedBlocks;
  return (int)g;
}

// Dense operator y_r = sc * sum_j X[j][.] b_r[j] (X row-major nd x nd, row j
// holding the operator's column j), in two deterministic stages.  j is cut
// into kDenseChunks * kDenseWaves sub-chunks; block (64 outputs i, chunk c)
// of a launch for right-hand sides r0 .. r0 + NR - 1 has one wave per
// sub-chunk of chunk c, which sums it in j order with kDenseLoads rows of X
// in flight per lane (b read by scalar loads: the wave index is made
// wave-uniform so that the addresses are); the waves' sums are added in wave
// order through LDS into part[c][r][i].  The second stage adds the chunks in
// order and scales.  For nd = 4096 the first stage runs 16 waves per CU.
constexpr int kDenseWaves = 8;
constexpr int kDenseLoads = 16;
template <typename T, int NR>
__global__ void __launch_bounds__(64 * kDenseWaves)
k_dense_part(const T* __restrict__ X, int nd, const T* __restrict__ b, int nrhs, int r0, T* __restrict__ part) {
  __shared__ T red[kDenseWaves][NR][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ch = (nd + kDenseChunks * kDenseWaves - 1) / (kDenseChunks * kDenseWaves);
  const int j0 = (blockIdx.y * kDenseWaves + w) * ch;
  const int len = (j0 >= nd) ? 0 : (nd - j0 < ch ? nd - j0 : ch);
  const int i = blockIdx.x * 64 + lane;
  const T* __restrict__ xp = X + (long long)j0 * nd + (i < nd ? i : 0);
  const T* __restrict__ bp = b + (long long)r0 * nd + j0;
  T acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = T(0);
  int jj = 0;
  for (; jj + kDenseLoads <= len; jj += kDenseLoads) {
    T xv[kDenseLoads];
#pragma unroll
    for (int u = 0; u < kDenseLoads; ++u) xv[u] = xp[(long long)(jj + u) * nd];
#pragma unroll
    for (int u = 0; u < kDenseLoads; ++u)
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] += xv[u] * bp[(long long)r * nd + jj + u];
  }
  for (; jj < len; ++jj) {
    const T xv = xp[(long long)jj * nd];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] += xv * bp[(long long)r * nd + jj];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) red[w][r][lane] = acc[r];
  __syncthreads();
  const int r = threadIdx.x >> 6;
  if (r < NR && i < nd) {
    T sum = red[0][r][lane];
#pragma unroll
    for (int v = 1; v < kDenseWaves; ++v) sum += red[v][r][lane];
    part[((long long)blockIdx.y * nrhs + r0 + r) * nd + i] = sum;
  }
}

// Matrix-core form of the first stage for 2..16 right-hand sides: the
// product (right-hand sides x matrix) in 16x16x4 MFMA steps, A = the 16
// right-hand sides' values at 4 consecutive j (zero past nrhs), B = 4 rows j
// of 16 matrix columns, so the matrix is read once for all right-hand sides.
// Block (64 columns i, chunk c) has one wave per j sub-chunk of chunk c, each
// accumulating four 16x16 tiles (right-hand side x column); the waves' tiles
// are added in wave order through LDS (two rounds of four waves) into
// part[c][r][i].  Lane l supplies A(l % 16, l / 16) and B(l / 16, l % 16) and
// receives D(row, l % 16) in element v < 4 with row = l / 16 + 4 v for the
// FP64 instruction and 4 (l / 16) + v for the FP32 one (checked on gfx950).
typedef double dense_f64x4 __attribute__((ext_vector_type(4)));
typedef float dense_f32x4 __attribute__((ext_vector_type(4)));
template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  using V = dense_f64x4;
  static __device__ __forceinline__ V step(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int kq, int v) { return kq + 4 * v; }
};
template <>
struct MfmaAcc<float> {
  using V = dense_f32x4;
  static __device__ __forceinline__ V step(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ constexpr int row(int kq, int v) { return 4 * kq + v; }
};
constexpr int kDenseSteps = 4;  // MFMA steps (4 j each) whose loads are issued together
template <typename T>
__global__ void __launch_bounds__(64 * kDenseWaves)
k_dense_mfma(const T* __restrict__ X, int nd, const T* __restrict__ b, int nrhs, T* __restrict__ part) {
  using V = typename MfmaAcc<T>::V;
  __shared__ T red[kDenseWaves / 2][16][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = lane & 15, kq = lane >> 4;
  int ch = (nd + kDenseChunks * kDenseWaves - 1) / (kDenseChunks * kDenseWaves);
  ch = (ch + 3) & ~3;
  const int j0 = (blockIdx.y * kDenseWaves + w) * ch;
  const int j1 = (j0 + ch < nd) ? j0 + ch : nd;
  const int c0 = blockIdx.x * 64;
  const bool rok = col < nrhs;
  const T* __restrict__ bp = b + (long long)(rok ? col : 0) * nd;
  bool cok[4];
  const T* __restrict__ xp[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i = c0 + 16 * t + col;
    cok[t] = i < nd;
    xp[t] = X + (cok[t] ? i : 0);
  }
  V acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = V{};
  for (int jj = j0; jj < j1; jj += 4 * kDenseSteps) {
    T av[kDenseSteps], bv[kDenseSteps][4];
#pragma unroll
    for (int u = 0; u < kDenseSteps; ++u) {
      const int j = jj + 4 * u + kq;
      const bool jok = j < j1;
      av[u] = (jok && rok) ? bp[j] : T(0);
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[u][t] = (jok && cok[t]) ? xp[t][(long long)j * nd] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kDenseSteps; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = MfmaAcc<T>::step(av[u], bv[u][t], acc[t]);
  }
  // waves 0..3, then 4..7, added in wave order
  const int tr = threadIdx.x >> 6, tc = threadIdx.x & 63;  // this thread's outputs: rows tr, tr + 8
  T sum[2] = {T(0), T(0)};
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if (w / 4 == half)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[w % 4][MfmaAcc<T>::row(kq, v)][16 * t + col] = acc[t][v];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T x = red[v][tr + 8 * e][tc];
        sum[e] = (half == 0 && v == 0) ? x : sum[e] + x;
      }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int r = tr + 8 * e, i = c0 + tc;
    if (r < nrhs && i < nd) part[((long long)blockIdx.y * nrhs + r) * nd + i] = sum[e];
  }
}

template <typename T, int NR>
void launch_dense_part(const T* X, int nd, const T* b, int nrhs, int r0, T* part, hipStream_t s) {
  const dim3 g((nd + 63) / 64, kDenseChunks);
  hipLaunchKernelGGL((k_dense_part<T, NR>), g, dim3(64 * kDenseWaves), 0, s, X, nd, b, nrhs, r0, part);
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_dense_sum(const T* __restrict__ part, int nd, int nrhs, T sc, T* __restrict__ y) {
  const int i = blockIdx.x * kRedThreads + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= nd) return;
  T sum = T(0);
  for (int c = 0; c < kDenseChunks; ++c) sum += part[((long long)c * nrhs + r) * nd + i];
  y[(long long)r * nd + i] = sc * sum;
}

// b[r][i] = (i == r0 + r): a batch of unit vectors
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_unit_batch(T* __restrict__ b, int nd, int r0) {
  const int i = blockIdx.x * kRedThreads + threadIdx.x;
  const int r = blockIdx.y;
  if (i < nd) b[(long long)r * nd + i] = (i == r0 + r) ? T(1) : T(0);
}

}  // namespace

hipError_t blas_dot2(const double* a, const double* b, const double* c, const double* d,
                     long long n, int nrhs, double* partial, double* partial2, double* out,
                     double* out2, hipStream_t s) {
  const int g = grid_for(n);
  hipLaunchKernelGGL(k_dot2<double>, dim3(g, nrhs), dim3(kRedThreads), 0, s, a, b, c, d, n, n, n, partial,
                     partial2);
  if (out) hipLaunchKernelGGL(k_finalize, dim3(nrhs), dim3(kRedThreads), 0, s, partial, g, out);
  if (c && out2) hipLaunchKernelGGL(k_finalize, dim3(nrhs), dim3(kRedThreads), 0, s, partial2, g, out2);
  return hipGetLastError();
}

hipError_t blas_neg_finalize_sum(const double* partial, long long n, int nrhs, double* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_neg_finalize, dim3(nrhs), dim3(kRedThreads), 0, s, partial, grid_for(n), out);
  hipLaunchKernelGGL(k_sum_rhs, dim3(1), dim3(64), 0, s, out, nrhs);
  return hipGetLastError();
}

hipError_t blas_multi_dot(const double* V, const double* w, long long n, int m, double* partial,
                          double* out, hipStream_t s) {
  const int g = grid_for(n);
  hipLaunchKernelGGL(k_dot2<double>, dim3(g, m), dim3(kRedThreads), 0, s, V, w, nullptr, nullptr, n, n, 0LL,
                     partial, nullptr);
  hipLaunchKernelGGL(k_finalize, dim3(m), dim3(kRedThreads), 0, s, partial, g, out);
  return hipGetLastError();
}

hipError_t blas_multi_axpy(double* w, const double* V, const double* coef, int m, double sgn,
                           long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_multi_axpy, dim3(grid_for(n)), dim3(kRedThreads), 0, s, w, V, coef, m, sgn, n);
  return hipGetLastError();
}

hipError_t blas_normalise(double* v, double* v2, const double* w, const double* nn, long long n,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_normalise, dim3(grid_for(n)), dim3(kRedThreads), 0, s, v, v2, w, nn, n);
  return hipGetLastError();
}

hipError_t blas_update_xr(double* x, double* r, const double* p, const double* q, const double* rz,
                          const double* pq_part, double* pq, const int* active, long long n,
                          int nrhs, double* alpha, double* partial, float* r32, hipStream_t s) {
  const int g = grid_for(n);
  hipLaunchKernelGGL(k_update_xr, dim3(g, nrhs), dim3(kRedThreads), 0, s, x, r, p, q, rz, pq_part, g,
                     pq, active, n, alpha, partial, r32);
  return hipGetLastError();
}

hipError_t blas_cg_check(const double* rr_part, long long n, int nrhs, double* rr, const double* pq,
                         const double* nb, double rtol, int* active, double* rec, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_check, dim3(nrhs), dim3(kRedThreads), 0, s, rr_part, grid_for(n), rr, pq,
                     nb, rtol, active, rec);
  return hipGetLastError();
}

hipError_t blas_update_p(double* p, const double* z, const double* rz_part, const double* zq_part,
                         double* rz_new, double* zq, const double* rz_old, const double* alpha,
                         const int* active, int flexible, long long n, int nrhs, hipStream_t s) {
  const int g = grid_for(n);
  hipLaunchKernelGGL(k_update_p<double>, dim3(g, nrhs), dim3(kRedThreads), 0, s, p, z, rz_part, zq_part,
                     g, rz_new, zq, rz_old, alpha, active, flexible, n);
  return hipGetLastError();
}

hipError_t blas_finalize(const double* partial, long long n, int nrhs, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(nrhs), dim3(kRedThreads), 0, s, partial, grid_for(n), out);
  return hipGetLastError();
}

hipError_t blas_dot2_z32(const double* r, const float* z, const float* zc, const double* q,
                         long long n, int nrhs, double* partial, double* partial2, hipStream_t s) {
  hipLaunchKernelGGL(k_dot2<float>, dim3(grid_for(n), nrhs), dim3(kRedThreads), 0, s, r, z, zc, q, n,
                     n, n, partial, partial2);
  return hipGetLastError();
}

hipError_t blas_update_p_z32(double* p, const float* z, const double* rz_part, const double* zq_part,
                             double* rz_new, double* zq, const double* rz_old, const double* alpha,
                             const int* active, int flexible, long long n, int nrhs, hipStream_t s) {
  const int g = grid_for(n);
  hipLaunchKernelGGL(k_update_p<float>, dim3(g, nrhs), dim3(kRedThreads), 0, s, p, z, rz_part, zq_part,
                     g, rz_new, zq, rz_old, alpha, active, flexible, n);
  return hipGetLastError();
}

hipError_t blas_f64_to_f32(const double* a, float* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_for(n)), dim3(kRedThreads), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t blas_f32_to_f64(const float* a, double* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(n)), dim3(kRedThreads), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t blas_zero_f64(double* a, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(n)), dim3(kRedThreads), 0, s, a, 0.0, n);
  return hipGetLastError();
}

hipError_t blas_zero_f32(float* a, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_fill<float>), dim3(grid_for(n)), dim3(kRedThreads), 0, s, a, 0.0f, n);
  return hipGetLastError();
}

template <typename T>
hipError_t dense_apply(const T* X, int nd, const T* b, T* y, int nrhs, T sc, T* part, hipStream_t s) {
  if (nd <= 0 || nrhs <= 0) return hipErrorInvalidValue;
  if (nrhs > 1 && nrhs <= 16) {
    const dim3 g((nd + 63) / 64, kDenseChunks);
    hipLaunchKernelGGL((k_dense_mfma<T>), g, dim3(64 * kDenseWaves), 0, s, X, nd, b, nrhs, part);
  } else
  for (int r0 = 0; r0 < nrhs; r0 += kDenseRhs) {
    switch (nrhs - r0 < kDenseRhs ? nrhs - r0 : kDenseRhs) {
      case 1: launch_dense_part<T, 1>(X, nd, b, nrhs, r0, part, s); break;
      case 2: launch_dense_part<T, 2>(X, nd, b, nrhs, r0, part, s); break;
      case 3: launch_dense_part<T, 3>(X, nd, b, nrhs, r0, part, s); break;
      case 4: launch_dense_part<T, 4>(X, nd, b, nrhs, r0, part, s); break;
      case 5: launch_dense_part<T, 5>(X, nd, b, nrhs, r0, part, s); break;
      case 6: launch_dense_part<T, 6>(X, nd, b, nrhs, r0, part, s); break;
      case 7: launch_dense_part<T, 7>(X, nd, b, nrhs, r0, part, s); break;
      default: launch_dense_part<T, 8>(X, nd, b, nrhs, r0, part, s); break;
    }
  }
  const dim3 g2((nd + kRedThreads - 1) / kRedThreads, nrhs);
  hipLaunchKernelGGL((k_dense_sum<T>), g2, dim3(kRedThreads), 0, s, part, nd, nrhs, sc, y);
  return hipGetLastError();
}
template hipError_t dense_apply<double>(const double*, int, const double*, double*, int, double, double*,
                                        hipStream_t);
template hipError_t dense_apply<float>(const float*, int, const float*, float*, int, float, float*, hipStream_t);

template <typename T>
hipError_t unit_batch(T* b, int nd, int r0, int count, hipStream_t s) {
  const dim3 g((nd + kRedThreads - 1) / kRedThreads, count);
  hipLaunchKernelGGL((k_unit_batch<T>), g, dim3(kRedThreads), 0, s, b, nd, r0);
  return hipGetLastError();
}
template hipError_t unit_batch<double>(double*, int, int, int, hipStream_t);
template hipError_t unit_batch<float>(float*, int, int, int, hipStream_t);

hipError_t blas_sub(const double* a, const double* b, double* y, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(grid_for(n)), dim3(kRedThreads), 0, s, a, b, y, n);
  return hipGetLastError();
}

}  // namespace dgmg
