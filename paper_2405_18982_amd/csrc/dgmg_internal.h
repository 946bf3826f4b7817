// Internal declarations shared by the host orchestration (dgmg_api.cpp) and
// the per-(dimension, degree) kernel translation units (dgmg_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgmg {

constexpr int kMaxDegree = 7;
constexpr int kMaxLevels = 21;   // levels 0..20 (finest level L <= 20)
// workgroup shapes of apply: 0, 1 patches per workgroup; 2 face data in
// registers; 3 several right-hand sides of one patch per workgroup
constexpr int kApplyShapes = 4;
// workgroup shapes of the smoother: 0..7 patches per workgroup x prefetch of
// b x (two waves per patch | one patch per workgroup); 8..11 several
// right-hand sides of one patch per workgroup (two slot counts) x prefetch
constexpr int kSmoothShapes = 12;

// Reference (h = 1, kappa = 1) data of Q_K on a two-cell patch that depends
// on the penalty, in the arithmetic type T of the kernels that read them.
// Built on the host in FP64 (setup.cpp) and uploaded once per context.  (The
// basis matrices that depend on K alone -- mass, stiffness, end derivatives,
// prolongation -- are compile-time constants, dgmg_ref1d.h.)
//   sigma : penalty factor (gamma_F = sigma / h)
//   S[t], lam[t] : fast-diagonalisation eigenpairs of patch type t on the
//         Dirichlet local space, padded to E (unused eigenvalue slots hold a
//         huge finite value)
//   Sf[t], lamf[t] : the same on the whole patch (Full kernel)
//   Sc[t], lamc[t] : C S on the clamped space with basis C (clamped kernel)
//   rs[s][c] : the inverse eigenvalue sums of the fast-diagonalisation solve
//         of local space s (0 Dirichlet, 1 whole patch, 2 clamped) for the
//         patch-type combination c, computed in FP64 and rounded: in 3-D,
//         c = (tx 4 + ty) 4 + tz and rs[s][c][(qz E + qx) E + qy] =
//         1 / (lam_y[qy] + (lam_x[qx] + lam_z[qz])); in 2-D, c = tx 4 + ty and
//         rs[s][c][qy E + qx] = 1 / (lam_x[qx] + lam_y[qy]); 0 where a slot is
//         unused
template <int K, typename T>
struct Tab {
  static constexpr int n = K + 1;
  static constexpr int E = 2 * n;
  T sigma;
  T S[4][E * E];
  T lam[4][E];
  T Sf[4][E * E];
  T lamf[4][E];
  T Sc[4][E * E];
  T lamc[4][E];
  T rs[3][64][E * E * E];
};

// The patches of one launch: patch m = (m_0, .., m_{D-1}), m_i < cnt[i], has
// its lower-left cell at lo_i = off[i] + 2 m_i and covers cells lo_i, lo_i + 1.
// The Full smoother's launches also carry the partial patches that complete
// the tiling of the mesh (off = -1: lo_i = -1 or N - 1, one cell inside).
struct PatchGrid {
  int N;       // cells per direction on the level
  int cnt[3];  // patches per direction
  int off[3];  // -1, 0 or 1
  int npatch;  // product of cnt
  int xcd_remap;  // 1: give each XCD a contiguous range of patches
  int nrhs;    // right-hand sides of the launch (set by the launchers)
};

// Host-visible launchers of one (D, K) instantiation.  All vectors are
// [nrhs][ndof] device arrays; `tab` points to a device Tab<K, T>.
template <typename T>
struct KernelSet {
  // apply and smooth come in several tuned shapes (patches per workgroup; for
  // the smoother also whether b is prefetched)
  hipError_t (*apply[kApplyShapes])(const void* tab, PatchGrid g, T scale, const T* x, T* y, int nrhs,
                         long long ndof, hipStream_t s);
  // 1 where apply shape 2 (face data in registers) differs from shape 0
  int apply_rf;
  // 1 where the right-hand-side-packed shapes (apply 3, smoother 8..11) hold
  // more than one slot per workgroup
  int apply_rpack;
  int smooth_rpack;
  hipError_t (*mass)(const void* tab, PatchGrid g, T scale, const T* x, T* y, int nrhs,
                     long long ndof, hipStream_t s);
  // variant: DGMG_SMOOTH_* of the context.  The Dirichlet kernels update x in
  // place (xin is ignored); the Full kernel reads xin and writes xout.  zero:
  // colour 0 of a step that starts from x = 0 (x is not read, every node of
  // xout is written).
  hipError_t (*smooth[kSmoothShapes])(const void* tab, PatchGrid g, T scale, T inv_scale, int variant,
                          int zero, const T* xin, T* xout, const T* b, int nrhs, long long ndof,
                          hipStream_t s);
  // 1 where shapes 4..7 (two waves per patch, or one patch per workgroup
  // where patches share a wave) differ from 0..3; smooth_hi_full: also for
  // the Full kernel
  int smooth_split;
  int smooth_hi_full;
  hipError_t (*restrict_residual)(const void* tab, PatchGrid g, T scale, const T* x, const T* b,
                                  T* bc, int nrhs, long long ndof, long long ndof_c,
                                  hipStream_t s);
  hipError_t (*prolongate_add)(const void* tab, PatchGrid g, const T* xc, T* x, int nrhs,
                               long long ndof, long long ndof_c, hipStream_t s);
  hipError_t (*coarse)(const void* tab, T inv_scale, const T* b, T* x, int nrhs,
                       long long ndof, hipStream_t s);
  // levels 1 and 0 of the V-cycle in one launch (pre-smoothing from zero,
  // restriction, coarse solve, prolongation, post-smoothing); null where the
  // level-1 patches of a colour do not fit one workgroup
  // (split: two waves per patch in the smoothing stages, where bottom_split)
  hipError_t (*bottom)(const void* tab, int variant, int split, T scale1, T inv_scale1, T inv_scale0,
                       T* x1, const T* b1, T* b0, T* x0, int nrhs, long long ndof1, long long ndof0,
                       hipStream_t s);
  int bottom_split;
  // 2-D: levels 2, 1 and 0 in one launch (null where they do not fit)
  hipError_t (*bottom3)(const void* tab, int variant, T scale2, T inv_scale2, T scale1, T inv_scale1,
                        T inv_scale0, T* x2, const T* b2, T* x1, T* b1, T* b0, T* x0, int nrhs,
                        long long ndof2, long long ndof1, long long ndof0, hipStream_t s);
};

// Registration entry of one kernel translation unit.
struct KernelEntry {
  int dim;
  int degree;
  KernelSet<double> f64;
  KernelSet<float> f32;
};

}  // namespace dgmg

// Each kernel TU defines dgmg_kernels_d<D>_k<K>(KernelEntry*).
#define DGMG_KERNEL_ENTRY_NAME(D, K) dgmg_kernels_d##D##_k##K
#define DGMG_DECLARE_ENTRY(D, K) \
  extern "C" void DGMG_KERNEL_ENTRY_NAME(D, K)(dgmg::KernelEntry * e);
