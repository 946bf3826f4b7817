// Vector kernels of the outer Krylov iteration (dgmg_blas.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace dgmg {

// Upper bound of the first-stage blocks per right-hand side of a reduction;
// partial-sum buffers hold nrhs * kRedBlocks doubles.
constexpr int kRedBlocks = 1024;

// out[r] = a_r . b_r (and out2[r] = c_r . d_r when c != nullptr), vectors
// [nrhs][n]; deterministic for given (n, nrhs).  out == nullptr (out2 ==
// nullptr): only the first-stage partial sums, which the consuming kernel
// finishes itself (the same value bit for bit).
hipError_t blas_dot2(const double* a, const double* b, const double* c, const double* d,
                     long long n, int nrhs, double* partial, double* partial2, double* out,
                     double* out2, hipStream_t s);
// CG update x += alpha p, r -= alpha q, alpha = rz / pq per active right-hand
// side, with p^T q finished from the partial sums pq_part of blas_dot2 (and
// stored to pq); partial: first-stage sums of |r|^2 (must not alias pq_part).
// r32 != nullptr: also r32 = (float) r for the active right-hand sides.
hipError_t blas_update_xr(double* x, double* r, const double* p, const double* q, const double* rz,
                          const double* pq_part, double* pq, const int* active, long long n,
                          int nrhs, double* alpha, double* partial, float* r32, hipStream_t s);
// rr = |r|^2 from rr_part; active &&= sqrt(rr) / nb > rtol; rec (device
// address of host-visible memory, 4 doubles per right-hand side) =
// (rr, pq, sqrt(rr) / nb, active).
hipError_t blas_cg_check(const double* rr_part, long long n, int nrhs, double* rr, const double* pq,
                         const double* nb, double rtol, int* active, double* rec, hipStream_t s);
// p = z + beta p per active right-hand side, rz_new (and zq) finished from
// the partial sums of blas_dot2 and stored.
hipError_t blas_update_p(double* p, const double* z, const double* rz_part, const double* zq_part,
                         double* rz_new, double* zq, const double* rz_old, const double* alpha,
                         const int* active, int flexible, long long n, int nrhs, hipStream_t s);
// out[r] = sum of the first-stage partial sums that blas_dot2 left for
// vectors of length n (the second stage it skips when out == nullptr).
hipError_t blas_finalize(const double* partial, long long n, int nrhs, double* out, hipStream_t s);
// The same two steps with z the FP32 output of the V-cycle (its values taken
// exactly in FP64): partial sums of r^T z (and, zc = z, z^T q), and p update.
hipError_t blas_dot2_z32(const double* r, const float* z, const float* zc, const double* q,
                         long long n, int nrhs, double* partial, double* partial2, hipStream_t s);
hipError_t blas_update_p_z32(double* p, const float* z, const double* rz_part, const double* zq_part,
                             double* rz_new, double* zq, const double* rz_old, const double* alpha,
                             const int* active, int flexible, long long n, int nrhs, hipStream_t s);
// out[r] = -(sum of the first-stage partial sums blas_dot2 left for vectors
// of length n), r < nrhs, then out[nrhs] = sum_r out[r] (out: nrhs + 1
// doubles): the coefficient gradient -lambda^T A_1 u per right-hand side and
// in total.
hipError_t blas_neg_finalize_sum(const double* partial, long long n, int nrhs, double* out,
                                 hipStream_t s);
// out[i] = V_i . w for the m vectors V_i = V + i n (partial: m * kRedBlocks).
hipError_t blas_multi_dot(const double* V, const double* w, long long n, int m, double* partial,
                          double* out, hipStream_t s);
// w += sgn * sum_i coef[i] V_i (coef: device array of m doubles).
hipError_t blas_multi_axpy(double* w, const double* V, const double* coef, int m, double sgn,
                           long long n, hipStream_t s);
// v = w / sqrt(nn[0]), and the same into v2 unless it is null.
hipError_t blas_normalise(double* v, double* v2, const double* w, const double* nn, long long n,
                          hipStream_t s);
hipError_t blas_f64_to_f32(const double* a, float* b, long long n, hipStream_t s);
hipError_t blas_f32_to_f64(const float* a, double* b, long long n, hipStream_t s);
hipError_t blas_zero_f64(double* a, long long n, hipStream_t s);
hipError_t blas_zero_f32(float* a, long long n, hipStream_t s);
hipError_t blas_sub(const double* a, const double* b, double* y, long long n, hipStream_t s);

// Dense operator of the V-cycle's bottom levels: y_r = sc * sum_j X[j][.]
// b_r[j] for r < nrhs, X row-major nd x nd (row j = the operator's column j),
// b and y [nrhs][nd]; deterministic (fixed chunks summed in order, in T).
// part: kDenseChunks * nrhs * nd values of T.  One right-hand side (and
// more than 16, in groups of kDenseRhs): vector units; 2..16: matrix cores,
// X read once.
constexpr int kDenseChunks = 8;
constexpr int kDenseRhs = 8;
template <typename T>
hipError_t dense_apply(const T* X, int nd, const T* b, T* y, int nrhs, T sc, T* part, hipStream_t s);
// b[r][i] = (i == r0 + r) for r < count: unit vectors r0 .. r0 + count - 1
template <typename T>
hipError_t unit_batch(T* b, int nd, int r0, int count, hipStream_t s);

}  // namespace dgmg
