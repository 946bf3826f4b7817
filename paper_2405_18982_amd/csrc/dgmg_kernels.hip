// Patch-tile kernels of the SIPG multigrid hot path for one (dimension D,
// degree K) pair, selected by -DDGMG_D=<2|3> -DDGMG_K=<1..7>; the build
// compiles this file once per pair.
//
// Every kernel works on "patches": the 2^D cells with coordinates lo_i and
// lo_i + 1 in each direction i.  A patch carries E = 2(K+1) nodes per
// direction (patch-local index p = n c + a for cell c in {0,1}, node a).  A
// workgroup owns PPB patches, TPP = E^(D-1) threads each (one wave per patch
// for 3-D K <= 3, several 2-D patches per wave).  Work proceeds in phases
// separated by barriers; in a phase along direction `dir` each thread owns one
// 1-D line of the patch (all other coordinates fixed), contracts it in
// registers with the 1-D matrices (wave-uniform operands read through scalar
// loads from the Tab struct) and hands the result to the next phase through
// LDS.  The first phase (along x) reads its lines straight from global memory:
// an x-line of a patch is two contiguous cell rows, and its outside neighbours
// across the x-faces are the adjacent rows, so x itself never passes through
// LDS.  Smoothers keep that x-line in registers and finish with another
// x-phase that writes x + delta back as contiguous rows.
//
// Operator (Sec. 2.2): on a Cartesian mesh A = sum_i (x)(M .. L_i .. M), with
// reference matrices (h = 1) and A_h = kappa h^(D-2) A_ref.  The 1-D SIPG
// operator restricted to the patch is applied per cell block (Lc: both faces
// interior) plus rank-2 face terms e alpha + d beta:
//   interior face, neighbour on the left  (its x=1 side, trace t, derivative g):
//       alpha = g/2 - sigma t, beta = -t/2   on the rows e0, d0
//   interior face, neighbour on the right (its x=0 side):
//       alpha = -sigma t - g/2, beta = t/2   on the rows e1, d1
//   domain-boundary face (Nitsche), from the cell's own line v:
//       x=0: alpha = (d0.v)/2, beta = v_0/2;  x=1: alpha = -(d1.v)/2, beta = -v_k/2
// Face data of interior neighbours across y- and z-faces ("ext") is gathered
// per face node into LDS and contracted with the tangential masses on the fly,
// giving the sum-factorised order
//   a = M_x x, b = L_x x;  c = M_y b + L_y a, d = M_y a;  y = M_z c + L_z d.
#include "dgmg_internal.h"
#include "dgmg_ref1d.h"

#ifndef DGMG_D
#error "DGMG_D must be defined"
#endif
#ifndef DGMG_K
#error "DGMG_K must be defined"
#endif

// Multiply-adds are fused only within one expression (never across
// statements), so every kernel variant that writes an output with the same
// expressions -- one or two waves per patch, fused or separate launches --
// computes it bit for bit alike, whatever the surrounding control flow.
#pragma clang fp contract(on)

namespace dgmg {
namespace {

constexpr int D = DGMG_D;
constexpr int K = DGMG_K;
constexpr int n = K + 1;
constexpr int E = 2 * n;
constexpr int NL = (D == 2) ? E : E * E;            // lines per direction
constexpr int NC = (D == 2) ? n * n : n * n * n;    // nodes per cell
constexpr int NCP = (D == 2) ? 4 : 8;               // cells per patch
constexpr int SY = E + 1;                           // padded LDS strides
constexpr int SZ = (D == 3) ? E * SY : 0;
constexpr int TS = (D == 2) ? E * SY : E * SZ;      // padded tile size
constexpr int NF = (D == 2) ? E : E * E;            // nodes of one patch face

// Basis data of Q_K fixed at compile time (instruction immediates); only the
// penalty and the patch eigenpairs come from the Tab struct.
static constexpr ref1d::Ref<K> kRef = ref1d::make_ref<K>();

// threads per patch (one per line) and patches per workgroup
constexpr int TPP = NL;
static_assert(TPP == NL, "each thread owns exactly one line per phase");
constexpr int PPB_DEFAULT = (D == 3)
    ? (K == 1 ? 4 : 1)
    : (K == 1 ? 16 : K == 2 ? 10 : K == 3 ? 8 : K == 4 ? 6 : K == 5 ? 5 : 4);

// base offset and stride of LDS line l along direction dir
__device__ __forceinline__ void line_geom(int dir, int l, int& base, int& stride) {
  const int a = l % E, b = l / E;
  if (dir == 0) { base = a * SY + b * SZ; stride = 1; }
  else if (dir == 1) { base = a + b * SZ; stride = SY; }
  else { base = a + b * SY; stride = SZ; }
}

template <typename T>
struct Line { T v[E]; };

template <typename T>
__device__ __forceinline__ void load_line(const T* s, int base, int stride, Line<T>& L) {
#pragma unroll
  for (int p = 0; p < E; ++p) L.v[p] = s[base + p * stride];
}
template <typename T>
__device__ __forceinline__ void store_line(T* s, int base, int stride, const Line<T>& L) {
#pragma unroll
  for (int p = 0; p < E; ++p) s[base + p * stride] = L.v[p];
}

// Even-odd form of the cell blocks (from Q4 on).  M and the consistency
// block Lcons are symmetric under the reflection of a cell (mu -> n-1-mu,
// nu -> n-1-nu), so B w for a cell line w is formed from sums ve and
// differences vo of mirrored values: the even part e = A ve (+ the middle
// column times the middle value for odd n), the odd part d = Bo vo, outputs
// e + d and e - d at mirrored rows (and the middle row from ve for odd n),
// with A, Bo the half-sums and half-differences of mirrored columns.  Fewer
// multiply-adds: 48 instead of 64 for n = 8.
constexpr bool kEOC = (K >= 4);
constexpr int kHN = n / 2;
constexpr bool kOddN = (n % 2) == 1;
struct EOCell {
  double A[kHN * kHN];
  double Bo[kHN * kHN];
  double colm[kHN + 1];  // middle column (rows < kHN), odd n
  double rowm[kHN + 1];  // middle row (columns < kHN, then the diagonal), odd n
};
constexpr EOCell make_eo_cell(const double (&B)[n * n]) {
  EOCell r{};
  for (int mu = 0; mu < kHN; ++mu)
    for (int j = 0; j < kHN; ++j) {
      r.A[mu * kHN + j] = 0.5 * (B[mu * n + j] + B[mu * n + n - 1 - j]);
      r.Bo[mu * kHN + j] = 0.5 * (B[mu * n + j] - B[mu * n + n - 1 - j]);
    }
  if (kOddN) {
    for (int mu = 0; mu < kHN; ++mu) r.colm[mu] = B[mu * n + kHN];
    for (int j = 0; j < kHN; ++j) r.rowm[j] = B[kHN * n + j];
    r.rowm[kHN] = B[kHN * n + kHN];
  }
  return r;
}
static constexpr EOCell kEOM = make_eo_cell(kRef.M);
static constexpr EOCell kEOL = make_eo_cell(kRef.Lcons);

// bl = B w for the cell c of patch line v (MASS: B = M, else Lcons)
template <typename T, bool MASS>
__device__ __forceinline__ void cell_eo(const Line<T>& v, int c, T (&bl)[n]) {
  constexpr const EOCell& C = MASS ? kEOM : kEOL;
  T ve[kHN], vo[kHN];
#pragma unroll
  for (int j = 0; j < kHN; ++j) {
    ve[j] = v.v[c * n + j] + v.v[c * n + n - 1 - j];
    vo[j] = v.v[c * n + j] - v.v[c * n + n - 1 - j];
  }
#pragma unroll
  for (int mu = 0; mu < kHN; ++mu) {
    T se = T(0), so = T(0);
#pragma unroll
    for (int j = 0; j < kHN; ++j) se += T(C.A[mu * kHN + j]) * ve[j];
    if constexpr (kOddN) se += T(C.colm[mu]) * v.v[c * n + kHN];
#pragma unroll
    for (int j = 0; j < kHN; ++j) so += T(C.Bo[mu * kHN + j]) * vo[j];
    bl[mu] = se + so;
    bl[n - 1 - mu] = se - so;
  }
  if constexpr (kOddN) {
    T sm = T(0);
#pragma unroll
    for (int j = 0; j < kHN; ++j) sm += T(C.rowm[j]) * ve[j];
    sm += T(C.rowm[kHN]) * v.v[c * n + kHN];
    bl[kHN] = sm;
  }
}

// o = blockdiag(M, M) v; the end outputs o[0] and o[E-1] only when need0 /
// needE (wave-uniform): smoothers drop them on interior patch faces
template <typename T>
__device__ __forceinline__ void line_mass(const Tab<K, T>* __restrict__ t, const Line<T>& v, Line<T>& o,
                                          bool need0 = true, bool needE = true) {
  if constexpr (kEOC) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      T bl[n];
      cell_eo<T, true>(v, c, bl);
#pragma unroll
      for (int mu = 0; mu < n; ++mu) {
        const int p = c * n + mu;
        if ((p == 0 && !need0) || (p == E - 1 && !needE)) continue;
        o.v[p] = bl[mu];
      }
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int mu = 0; mu < n; ++mu) {
      const int p = c * n + mu;
      if ((p == 0 && !need0) || (p == E - 1 && !needE)) continue;
      T s = T(0);
#pragma unroll
      for (int nu = 0; nu < n; ++nu) s += T(kRef.M[mu * n + nu]) * v.v[c * n + nu];
      o.v[p] = s;
    }
}

// 1/x from the hardware reciprocal estimate refined by one Newton step
// r <- r (2 - x r); the squared relative error of the estimate is far below
// the FP64 tolerance of the smoother.  x is a positive finite sum of patch
// eigenvalues (unused slots carry a huge finite value, giving ~0).
__device__ __forceinline__ double recip(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// Couplings of a patch line to what lies beyond its two outer faces.
template <typename T>
struct Sides {
  bool bl, br;   // left / right outer face on the domain boundary (Nitsche)
  T aL, bL, aR, bR;  // interior-neighbour couplings (ignored on boundary sides)
  // the paper's Dirichlet residual: on interior outer faces leave out the
  // consistency term -[[u]].{grad v} altogether (its inside half, carried by
  // the cell block, is cancelled from the line's own end value)
  bool lit;
};

// o (+)= 1-D SIPG of the patch line v; the end outputs only when need0 / needE
template <typename T, bool ACC>
__device__ __forceinline__ void line_sipg(const Tab<K, T>* __restrict__ t, const Line<T>& v,
                                          const Sides<T>& sd, Line<T>& o, bool need0 = true,
                                          bool needE = true) {
  const T sg = t->sigma;
  const T half = T(0.5);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    T bl[n];
    if constexpr (kEOC) cell_eo<T, false>(v, c, bl);
#pragma unroll
    for (int mu = 0; mu < n; ++mu) {
      const int p = c * n + mu;
      if ((p == 0 && !need0) || (p == E - 1 && !needE)) continue;
      T s = ACC ? o.v[p] : T(0);
      if constexpr (kEOC) {
        s += bl[mu];
      } else {
#pragma unroll
        for (int nu = 0; nu < n; ++nu) s += T(kRef.Lcons[mu * n + nu]) * v.v[c * n + nu];
      }
      if (mu == 0) s += sg * v.v[c * n];          // penalty part of the cell block
      if (mu == n - 1) s += sg * v.v[c * n + n - 1];
      o.v[p] = s;
    }
  }
  // face between the two patch cells
  const T tR = v.v[n];      // trace of the right cell at its x=0 side
  const T tL = v.v[n - 1];  // trace of the left cell at its x=1 side
  T gR = T(0), gL = T(0);
#pragma unroll
  for (int j = 0; j < n; ++j) {
    gR += T(kRef.d0[j]) * v.v[n + j];
    gL += T(kRef.d1[j]) * v.v[j];
  }
  T aL = sd.aL, bL = sd.bL, aR = sd.aR, bR = sd.bR;
  if (sd.bl) {  // Nitsche correction of the left cell (uniform per patch)
    T g0 = T(0);
#pragma unroll
    for (int j = 0; j < n; ++j) g0 += T(kRef.d0[j]) * v.v[j];
    aL = half * g0;
    bL = half * v.v[0];
  }
  if (sd.br) {
    T g1 = T(0);
#pragma unroll
    for (int j = 0; j < n; ++j) g1 += T(kRef.d1[j]) * v.v[n + j];
    aR = -half * g1;
    bR = -half * v.v[E - 1];
  }
  if (!sd.bl && sd.lit) bL = -half * v.v[0];
  if (!sd.br && sd.lit) bR = half * v.v[E - 1];
  const T bLc = half * tR;   // beta seen by the left cell from its right neighbour
  const T bRc = -half * tL;  // beta seen by the right cell from its left neighbour
  if (need0) {
    o.v[0] += aL;
    o.v[0] += T(kRef.d0[0]) * bL + T(kRef.d1[0]) * bLc;
  }
  o.v[n - 1] += -sg * tR - half * gR;
  o.v[n] += half * gL - sg * tL;
  if (needE) {
    o.v[E - 1] += aR;
    o.v[E - 1] += T(kRef.d0[n - 1]) * bRc + T(kRef.d1[n - 1]) * bR;
  }
#pragma unroll
  for (int mu = 0; mu < n; ++mu) {
    if (mu > 0) o.v[mu] += T(kRef.d0[mu]) * bL + T(kRef.d1[mu]) * bLc;
    if (mu < n - 1) o.v[n + mu] += T(kRef.d0[mu]) * bRc + T(kRef.d1[mu]) * bR;
  }
}

// Fast-diagonalisation contractions for patch type TY of a local space SP:
// SP_DIR the Dirichlet space, SP_FULL the whole patch, SP_CLAMPED the clamped
// space (tables C S).  Padded S: rows p in [PLO, PHI) and columns q < QN are
// the only non-zeros.
constexpr int SP_DIR = 0, SP_FULL = 1, SP_CLAMPED = 2;
template <int SP, int TY> struct FDB;
template <> struct FDB<SP_DIR, 0> { static constexpr int PLO = 1, PHI = E - 1, QN = E - 2; };
template <> struct FDB<SP_DIR, 1> { static constexpr int PLO = 0, PHI = E - 1, QN = E - 1; };
template <> struct FDB<SP_DIR, 2> { static constexpr int PLO = 1, PHI = E, QN = E - 1; };
template <> struct FDB<SP_DIR, 3> { static constexpr int PLO = 0, PHI = E, QN = E; };
template <int TY> struct FDB<SP_FULL, TY> { static constexpr int PLO = 0, PHI = E, QN = E; };
// clamped: value and derivative fixed at each interior-face end (two
// unknowns fewer per clamped end; the end node itself stays zero)
template <> struct FDB<SP_CLAMPED, 0> { static constexpr int PLO = 1, PHI = E - 1, QN = E - 4; };
template <> struct FDB<SP_CLAMPED, 1> { static constexpr int PLO = 0, PHI = E - 1, QN = E - 2; };
template <> struct FDB<SP_CLAMPED, 2> { static constexpr int PLO = 1, PHI = E, QN = E - 2; };
template <> struct FDB<SP_CLAMPED, 3> { static constexpr int PLO = 0, PHI = E, QN = E; };

template <typename T, int SP>
__device__ __forceinline__ const T* fd_S(const Tab<K, T>* __restrict__ t, int ty) {
  return SP == SP_FULL ? t->Sf[ty] : SP == SP_CLAMPED ? t->Sc[ty] : t->S[ty];
}
template <typename T, int SP>
__device__ __forceinline__ const T* fd_lam(const Tab<K, T>* __restrict__ t, int ty) {
  return SP == SP_FULL ? t->lamf[ty] : SP == SP_CLAMPED ? t->lamc[ty] : t->lam[ty];
}
// Inverse eigenvalue sums of the scaling line of a lane (3-D: the y-line
// (qx, qz) = (l % E, l / E); 2-D: the x-line qy = l): E values from the
// patch-type combination's table, read at the start of a colour step so that
// the loads overlap the operator passes.
template <typename T, int SP>
__device__ __forceinline__ void load_rs(const Tab<K, T>* __restrict__ t, const int (&ty)[3], int l,
                                        T (&r)[E]) {
  const int combo = (D == 3) ? (ty[0] * 4 + ty[1]) * 4 + ty[2] : ty[0] * 4 + ty[1];
  const T* p = t->rs[SP == SP_FULL ? 1 : SP == SP_CLAMPED ? 2 : 0][combo] + l * E;
#pragma unroll
  for (int q = 0; q < E; ++q) r[q] = p[q];
}

// Interior patches (type 0) on the Dirichlet space: the 1-D problem is
// symmetric under the reflection p -> E-1-p, and the host computes its
// eigenvectors on the even and the odd subspace (columns q < h even,
// h <= q < 2h odd, h = n - 1).  S^T then contracts sums v+ and differences v-
// of mirrored nodes with half columns, and S forms the even part e and odd
// part d of each mirrored pair: 2 h^2 multiply-adds instead of 4 h^2.  Used
// from Q4 on: measured on a smoothing step, 4-12% faster for Q4..Q7, 4-5%
// slower for Q3 (h = 3), where the dense contraction stays.
constexpr int kEOH = n - 1;
constexpr bool kEO = (K >= 4);

template <typename T>
__device__ __forceinline__ void eo_split(const Line<T>& v, T (&vp)[kEOH], T (&vm)[kEOH]) {
#pragma unroll
  for (int k = 0; k < kEOH; ++k) {
    vp[k] = v.v[1 + k] + v.v[E - 2 - k];
    vm[k] = v.v[1 + k] - v.v[E - 2 - k];
  }
}
// coefficient q < 2h of S^T v
template <typename T>
__device__ __forceinline__ T eo_coef(const T* S, const T (&vp)[kEOH], const T (&vm)[kEOH], int q) {
  T s = T(0);
#pragma unroll
  for (int k = 0; k < kEOH; ++k) s += S[(1 + k) * E + q] * (q < kEOH ? vp[k] : vm[k]);
  return s;
}
// even and odd parts of the outputs at nodes 1 + k and E - 2 - k of S v
template <typename T>
__device__ __forceinline__ void eo_pair(const T* S, const Line<T>& v, int k, T& e, T& d) {
  T se = T(0), sd = T(0);
#pragma unroll
  for (int q = 0; q < kEOH; ++q) se += S[(1 + k) * E + q] * v.v[q];
#pragma unroll
  for (int q = 0; q < kEOH; ++q) sd += S[(1 + k) * E + kEOH + q] * v.v[kEOH + q];
  e = se;
  d = sd;
}

// o[q] = sum_p S[p][q] v[p]
template <typename T, int TY, int SP>
__device__ __forceinline__ void line_St_t(const Tab<K, T>* __restrict__ t, const Line<T>& v, Line<T>& o) {
  using B = FDB<SP, TY>;
  const T* S = fd_S<T, SP>(t, TY);
  if constexpr (kEO && SP == SP_DIR && TY == 0) {
    T vp[kEOH], vm[kEOH];
    eo_split<T>(v, vp, vm);
#pragma unroll
    for (int q = 0; q < E; ++q) o.v[q] = (q < 2 * kEOH) ? eo_coef<T>(S, vp, vm, q) : T(0);
    return;
  }
#pragma unroll
  for (int q = 0; q < E; ++q) {
    T s = T(0);
    if (q < B::QN) {
#pragma unroll
      for (int p = B::PLO; p < B::PHI; ++p) s += S[p * E + q] * v.v[p];
    }
    o.v[q] = s;
  }
}
// o[p] = sum_q S[p][q] v[q]
template <typename T, int TY, int SP>
__device__ __forceinline__ void line_S_t(const Tab<K, T>* __restrict__ t, const Line<T>& v, Line<T>& o) {
  using B = FDB<SP, TY>;
  const T* S = fd_S<T, SP>(t, TY);
  if constexpr (kEO && SP == SP_DIR && TY == 0) {
    // outputs written in increasing node order, as in the other types: the
    // compiler then merges the four type branches' stores into one line
    // without a runtime-indexed copy of it (which would live in scratch)
    T e[kEOH], d[kEOH];
#pragma unroll
    for (int k = 0; k < kEOH; ++k) eo_pair<T>(S, v, k, e[k], d[k]);
    o.v[0] = T(0);
#pragma unroll
    for (int k = 0; k < kEOH; ++k) o.v[1 + k] = e[k] + d[k];
#pragma unroll
    for (int k = kEOH - 1; k >= 0; --k) o.v[E - 2 - k] = e[k] - d[k];
    o.v[E - 1] = T(0);
    return;
  }
#pragma unroll
  for (int p = 0; p < E; ++p) {
    T s = T(0);
    if (p >= B::PLO && p < B::PHI) {
#pragma unroll
      for (int q = 0; q < B::QN; ++q) s += S[p * E + q] * v.v[q];
    }
    o.v[p] = s;
  }
}
template <typename T, int SP>
__device__ __forceinline__ void line_St(const Tab<K, T>* __restrict__ t, int ty, const Line<T>& v, Line<T>& o) {
  switch (ty) {
    case 0: line_St_t<T, 0, SP>(t, v, o); break;
    case 1: line_St_t<T, 1, SP>(t, v, o); break;
    case 2: line_St_t<T, 2, SP>(t, v, o); break;
    default: line_St_t<T, 3, SP>(t, v, o); break;
  }
}
template <typename T, int SP>
__device__ __forceinline__ void line_S(const Tab<K, T>* __restrict__ t, int ty, const Line<T>& v, Line<T>& o) {
  switch (ty) {
    case 0: line_S_t<T, 0, SP>(t, v, o); break;
    case 1: line_S_t<T, 1, SP>(t, v, o); break;
    case 2: line_S_t<T, 2, SP>(t, v, o); break;
    default: line_S_t<T, 3, SP>(t, v, o); break;
  }
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Renumber them so that XCD j works on the j-th contiguous range of patches:
// neighbouring patches, whose face traces a patch reads, then sit in the
// same L2.  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_block(int b, int nblocks, int remap) {
  if (!remap || nblocks < 8) return b;
  const int q = nblocks / 8, r = nblocks % 8;
  const int xcd = b % 8, idx = b / 8;
  return xcd * q + (xcd < r ? xcd : r) + idx;
}

// Workgroup slot of the calling thread (TPP threads per slot): a scalar
// where a slot spans whole waves, so that the patch index and position that
// follow from it stay in scalar registers.
__device__ __forceinline__ int slot_of() {
  const int s = (int)threadIdx.x / TPP;
  if constexpr (TPP % 64 == 0) return __builtin_amdgcn_readfirstlane(s);
  return s;
}

// Patch and right-hand side of workgroup slot `slot`: PPB patches of one
// right-hand side per workgroup, or (RP, right-hand-side packing) one patch
// for PPB consecutive right-hand sides, so that every slot of the workgroup
// has the same patch type and position (uniform branches and scalar loads of
// the 1-D data where slots share a wave); slots past the last right-hand side
// get an out-of-range patch index and only meet the barriers.
template <int PPB, bool RP>
__device__ __forceinline__ void slot_work(const PatchGrid& g, int slot, int& pid, int& rhs) {
  const int blk = xcd_block(blockIdx.x, gridDim.x, g.xcd_remap);
  if constexpr (RP) {
    rhs = (int)blockIdx.y * PPB + slot;
    pid = rhs < g.nrhs ? blk : g.npatch;
    if (rhs >= g.nrhs) rhs = 0;
  } else {
    pid = blk * PPB + slot;
    rhs = blockIdx.y;
  }
}

// Patch coordinates of patch index pid of a launch.
struct PatchPos {
  int lo[3];
  int ty[3];  // 1-D patch type: bit 0 touches x_i = 0, bit 1 touches x_i = 1
};
__device__ __forceinline__ PatchPos patch_pos(const PatchGrid& g, int pid) {
  PatchPos P;
  int r = pid;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (i < D) {
      const int m = r % g.cnt[i];
      r /= g.cnt[i];
      P.lo[i] = g.off[i] + 2 * m;
      const int v = P.lo[i] + 1;  // the patch's vertex
      P.ty[i] = (v == 1 ? 1 : 0) | (v == g.N - 1 ? 2 : 0);
    } else {
      P.lo[i] = 0;
      P.ty[i] = 0;
    }
  }
  return P;
}

__device__ __forceinline__ long long cell_index(int N, int cx, int cy, int cz) {
  return (long long)cx + (long long)N * ((long long)cy + (long long)N * (long long)cz);
}

// Global offset of tile node (px, py, pz) of the patch.
__device__ __forceinline__ long long node_offset(int N, const PatchPos& P, int px, int py, int pz) {
  const int cx = px / n, ax = px % n;
  const int cy = py / n, ay = py % n;
  const int cz = (D == 3) ? pz / n : 0, az = (D == 3) ? pz % n : 0;
  const long long cell = cell_index(N, P.lo[0] + cx, P.lo[1] + cy, (D == 3) ? P.lo[2] + cz : 0);
  return cell * NC + ax + n * (ay + n * az);
}

// Global offset of the first node of the patch's x-line (py, pz) (cell lo_x).
__device__ __forceinline__ long long xrow_offset(int N, const PatchPos& P, int py, int pz) {
  return node_offset(N, P, 0, py, (D == 3) ? pz : 0);
}

// Side flags and x-face couplings of an x-line for the full operator from the
// n values of the rows of its outside x-neighbours (rl: the cell below, rr:
// the cell above; ignored on boundary sides).
template <typename T>
__device__ __forceinline__ Sides<T> xsides_rows(T sg, bool bl, bool br, const T (&rl)[n], const T (&rr)[n]) {
  const T half = T(0.5);
  Sides<T> sd;
  sd.bl = bl;
  sd.br = br;
  sd.aL = sd.bL = sd.aR = sd.bR = T(0);
  sd.lit = false;
  if (!sd.bl) {
    const T tr = rl[K];
    sd.bL = -half * tr;
    T g = T(0);
#pragma unroll
    for (int j = 0; j < n; ++j) g += T(kRef.d1[j]) * rl[j];
    sd.aL = half * g - sg * tr;
  }
  if (!sd.br) {
    const T tr = rr[0];
    sd.bR = half * tr;
    T g = T(0);
#pragma unroll
    for (int j = 0; j < n; ++j) g += T(kRef.d0[j]) * rr[j];
    sd.aR = -sg * tr - half * g;
  }
  return sd;
}

// Side flags and x-face couplings of x-line (py, pz), read from the rows of
// the outside neighbours.  MODE 0: full operator rows; 1: smoother (only the
// traces matter, alpha acts on dropped rows); 2: the paper's Dirichlet
// residual (interior neighbours ignored, consistency term left out).
template <typename T, int MODE>
__device__ __forceinline__ Sides<T> xline_sides(const Tab<K, T>* __restrict__ t, const T* __restrict__ x,
                                                int N, const PatchPos& P, long long row0) {
  const T half = T(0.5);
  const T sg = t->sigma;
  Sides<T> sd;
  sd.bl = (P.lo[0] == 0);
  sd.br = (P.lo[0] + 1 == N - 1);
  sd.aL = sd.bL = sd.aR = sd.bR = T(0);
  sd.lit = (MODE == 2);
  if (MODE != 2) {
    if (!sd.bl) {
      const T* r = x + row0 - NC;
      const T tr = r[K];
      sd.bL = -half * tr;
      if (MODE == 0) {
        T g = T(0);
#pragma unroll
        for (int j = 0; j < n; ++j) g += T(kRef.d1[j]) * r[j];
        sd.aL = half * g - sg * tr;
      }
    }
    if (!sd.br) {
      const T* r = x + row0 + 2 * NC;
      const T tr = r[0];
      sd.bR = half * tr;
      if (MODE == 0) {
        T g = T(0);
#pragma unroll
        for (int j = 0; j < n; ++j) g += T(kRef.d0[j]) * r[j];
        sd.aR = -sg * tr - half * g;
      }
    }
  }
  return sd;
}

// Raw face data of interior neighbours across y- (and z-) faces.  Entry i
// enumerates (dir, side, face node f); f = a + E b with (a, b) the tangential
// patch coordinates in increasing direction order.  NCOMP = 2 stores
// (alpha, beta), NCOMP = 1 stores beta only (MODE 2 stores zeros).  Layout: ext[(fd * 2 + side) *
// NCOMP + comp][f] with fd = dir - 1.
template <typename T, int MODE>
__device__ __forceinline__ void gather_ext(const Tab<K, T>* __restrict__ t, const T* __restrict__ x,
                                           int N, const PatchPos& P, int lane, T* ext) {
  constexpr int NCOMP = (MODE == 0) ? 2 : 1;
  constexpr int FD0 = (MODE == 0) ? 0 : 1;  // smoothers read y-face traces from global
  const T half = T(0.5);
  const T sg = t->sigma;
  // a patch face has one node per lane (NF = TPP), so entry block it = (fd -
  // FD0) * 2 + side holds this lane's face node f = lane: unrolled, direction
  // and side are compile-time constants of each block
  static_assert(NF == TPP, "one face node per lane");
#pragma unroll
  for (int it = 0; it < (D - 1 - FD0) * 2; ++it) {
    const int f = lane;
    const int side = it & 1;
    const int fd = it / 2 + FD0;
    const int dir = fd + 1;
    const int lod = (dir == 1) ? P.lo[1] : P.lo[2];  // not P.lo[dir]: no scratch copy of P
    const int nb = (side == 0) ? lod - 1 : lod + 2;
    T alpha = T(0), beta = T(0);
    if (MODE != 2 && nb >= 0 && nb < N) {
      // neighbour cell and the face node's local coordinates in it (tangential
      // coordinates from (a, b), 0 along dir); named per direction rather than
      // indexed by the runtime dir, which would put the arrays in scratch
      const int a = f % E, b = f / E;
      const int cx = P.lo[0] + a / n, ax = a % n;
      const int cy = (dir == 1) ? nb : P.lo[1] + b / n, ay = (dir == 1) ? 0 : b % n;
      const int cz = (D == 2) ? 0 : (dir == 1) ? P.lo[2] + b / n : nb;
      const int az = (D == 2 || dir != 1) ? 0 : b % n;
      const int strideN = (dir == 1) ? n : n * n;
      const long long base = cell_index(N, cx, cy, cz) * NC + ax + n * (ay + n * az);
      const T tr = x[base + (long long)((side == 0) ? K : 0) * strideN];
      beta = (side == 0) ? -half * tr : half * tr;
      if (MODE == 0) {
        T g = T(0);
#pragma unroll
        for (int j = 0; j < n; ++j) g += ((side == 0) ? T(kRef.d1[j]) : T(kRef.d0[j])) * x[base + (long long)j * strideN];
        alpha = (side == 0) ? (half * g - sg * tr) : (-sg * tr - half * g);
      }
    }
    if (NCOMP == 2) {
      ext[((fd * 2 + side) * 2 + 0) * NF + f] = alpha;
      ext[((fd * 2 + side) * 2 + 1) * NF + f] = beta;
    } else {
      ext[((fd - FD0) * 2 + side) * NF + f] = beta;
    }
  }
}

// row[nu] = M[mu][nu] for a lane-dependent mu, read from a device copy of
// the mass matrix (n vector loads instead of a select chain per entry)
template <typename T>
struct MassRows {
  T v[n * n];
};
template <typename T>
constexpr MassRows<T> make_mass_rows() {
  MassRows<T> r{};
  for (int i = 0; i < n * n; ++i) r.v[i] = T(kRef.M[i]);
  return r;
}
template <typename T>
__device__ constexpr MassRows<T> kMassRows = make_mass_rows<T>();

template <typename T>
__device__ __forceinline__ void mass_row(int mu, T (&row)[n]) {
#pragma unroll
  for (int nu = 0; nu < n; ++nu) row[nu] = kMassRows<T>.v[mu * n + nu];
}

// mass-contract ext entries along the first tangential coordinate for the
// value at (a, b): sum over the cell block of a
template <typename T>
__device__ __forceinline__ T ext_mx(const Tab<K, T>* __restrict__ t, const T* arr, int a, int b) {
  const int c0 = (a / n) * n, mu = a % n;
  T row[n];
  mass_row<T>(mu, row);
  T s = T(0);
#pragma unroll
  for (int nu = 0; nu < n; ++nu) s += row[nu] * arr[c0 + nu + E * b];
  return s;
}
template <typename T>
__device__ __forceinline__ T ext_my(const Tab<K, T>* __restrict__ t, const T* arr, int a, int b) {
  const int c0 = (b / n) * n, mu = b % n;
  T row[n];
  mass_row<T>(mu, row);
  T s = T(0);
#pragma unroll
  for (int nu = 0; nu < n; ++nu) s += row[nu] * arr[a + E * (c0 + nu)];
  return s;
}

// Sides of a y-line (px, pz) (D = 3) or (px) (D = 2): ext_y contracted with M_x.
template <typename T, int NCOMP>
__device__ __forceinline__ Sides<T> yline_sides(const Tab<K, T>* __restrict__ t, const T* ext,
                                                int N, const PatchPos& P, int px, int pz) {
  Sides<T> sd;
  sd.bl = (P.lo[1] == 0);
  sd.br = (P.lo[1] + 1 == N - 1);
  sd.aL = sd.bL = sd.aR = sd.bR = T(0);
  sd.lit = false;
  if (NCOMP == 2) {
    if (!sd.bl) { sd.aL = ext_mx<T>(t, ext + 0 * NF, px, pz); sd.bL = ext_mx<T>(t, ext + 1 * NF, px, pz); }
    if (!sd.br) { sd.aR = ext_mx<T>(t, ext + 2 * NF, px, pz); sd.bR = ext_mx<T>(t, ext + 3 * NF, px, pz); }
  } else {
    if (!sd.bl) sd.bL = ext_mx<T>(t, ext + 0 * NF, px, pz);
    if (!sd.br) sd.bR = ext_mx<T>(t, ext + 1 * NF, px, pz);
  }
  return sd;
}

// Sides of the smoother's y-line (px, pz): the traces of the y-neighbours at
// nodes (a, k or 0, pz), a in the cell block of px, contracted with M_x
// straight from global memory (n contiguous values per side).  MODE 2 (the
// paper's Dirichlet residual) ignores interior neighbours.  Split into the
// loads (yside_load: the mass row and both neighbours' n traces, the patch's
// own cells standing in for a missing neighbour, whose values go unused) and
// the arithmetic (yside_finish), so that callers can issue the loads together
// with their other global loads.
template <typename T>
struct YSideRaw {
  T row[n], l[n], r[n];
};
template <typename T, int MODE>
__device__ __forceinline__ void yside_load(const T* __restrict__ x, int N, const PatchPos& P, int px, int pz,
                                           YSideRaw<T>& y) {
  if (MODE == 2) return;
  const int cx = P.lo[0] + px / n;
  const int cz = (D == 3) ? P.lo[2] + pz / n : 0;
  const int az = (D == 3) ? pz % n : 0;
  const bool bl = (P.lo[1] == 0), br = (P.lo[1] + 1 == N - 1);
  mass_row<T>(px % n, y.row);
  const T* rl = x + cell_index(N, cx, bl ? P.lo[1] : P.lo[1] - 1, cz) * NC + K * n + az * n * n;
  const T* rr = x + cell_index(N, cx, br ? P.lo[1] + 1 : P.lo[1] + 2, cz) * NC + az * n * n;
#pragma unroll
  for (int nu = 0; nu < n; ++nu) {
    y.l[nu] = rl[nu];
    y.r[nu] = rr[nu];
  }
}
template <typename T, int MODE>
__device__ __forceinline__ Sides<T> yside_finish(const YSideRaw<T>& y, int N, const PatchPos& P) {
  Sides<T> sd;
  sd.bl = (P.lo[1] == 0);
  sd.br = (P.lo[1] + 1 == N - 1);
  sd.aL = sd.bL = sd.aR = sd.bR = T(0);
  sd.lit = (MODE == 2);
  if (MODE == 2) return sd;
  const T half = T(0.5);
  if (!sd.bl) {
    T s = T(0);
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += y.row[nu] * y.l[nu];
    sd.bL = -half * s;
  }
  if (!sd.br) {
    T s = T(0);
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += y.row[nu] * y.r[nu];
    sd.bR = half * s;
  }
  return sd;
}
// The same in one step (loads only the sides that exist, fewer live values).
template <typename T, int MODE>
__device__ __forceinline__ Sides<T> yline_sides_global(const Tab<K, T>* __restrict__ t,
                                                       const T* __restrict__ x, int N,
                                                       const PatchPos& P, int px, int pz) {
  Sides<T> sd;
  sd.bl = (P.lo[1] == 0);
  sd.br = (P.lo[1] + 1 == N - 1);
  sd.aL = sd.bL = sd.aR = sd.bR = T(0);
  sd.lit = (MODE == 2);
  if (MODE == 2) return sd;
  const int cx = P.lo[0] + px / n;
  const int cz = (D == 3) ? P.lo[2] + pz / n : 0;
  const int az = (D == 3) ? pz % n : 0;
  const T half = T(0.5);
  T row[n];
  if (!sd.bl || !sd.br) mass_row<T>(px % n, row);
  if (!sd.bl) {
    const T* r = x + cell_index(N, cx, P.lo[1] - 1, cz) * NC + K * n + az * n * n;
    T s = T(0);
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += row[nu] * r[nu];
    sd.bL = -half * s;
  }
  if (!sd.br) {
    const T* r = x + cell_index(N, cx, P.lo[1] + 2, cz) * NC + az * n * n;
    T s = T(0);
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += row[nu] * r[nu];
    sd.bR = half * s;
  }
  return sd;
}

// In the y-phase the z-face arrays are contracted along x in place (lines at
// fixed py); in the z-phase the value at (px, py) is contracted along y.
// z-face arrays follow the y-face arrays in the operator layout; smoothers
// keep only the z-face traces in LDS.
template <int NCOMP>
__device__ __forceinline__ constexpr int extz_base() { return NCOMP == 2 ? 4 * NF : 0; }

template <typename T, int NCOMP>
__device__ __forceinline__ void extz_mass_x_line(const Tab<K, T>* __restrict__ t, T* ext, int j) {
  const int py = j % E;
  const int arr = j / E;  // (side * NCOMP + comp)
  T* a = ext + extz_base<NCOMP>() + arr * NF + py * E;
  T v[E];
#pragma unroll
  for (int p = 0; p < E; ++p) v[p] = a[p];
  // dense mass rows (face data, contracted the same way wherever it is used)
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int mu = 0; mu < n; ++mu) {
      T s = T(0);
#pragma unroll
      for (int nu = 0; nu < n; ++nu) s += T(kRef.M[mu * n + nu]) * v[c * n + nu];
      a[c * n + mu] = s;
    }
}
template <typename T, int NCOMP>
__device__ __forceinline__ Sides<T> zline_sides(const Tab<K, T>* __restrict__ t, const T* ext,
                                                int N, const PatchPos& P, int px, int py) {
  Sides<T> sd;
  sd.bl = (P.lo[2] == 0);
  sd.br = (P.lo[2] + 1 == N - 1);
  sd.aL = sd.bL = sd.aR = sd.bR = T(0);
  sd.lit = false;
  const T* z = ext + extz_base<NCOMP>();
  if (NCOMP == 2) {
    if (!sd.bl) { sd.aL = ext_my<T>(t, z + 0 * NF, px, py); sd.bL = ext_my<T>(t, z + 1 * NF, px, py); }
    if (!sd.br) { sd.aR = ext_my<T>(t, z + 2 * NF, px, py); sd.bR = ext_my<T>(t, z + 3 * NF, px, py); }
  } else {
    if (!sd.bl) sd.bL = ext_my<T>(t, z + 0 * NF, px, py);
    if (!sd.br) sd.bR = ext_my<T>(t, z + 1 * NF, px, py);
  }
  return sd;
}

// zline_sides with NCOMP = 1 and the mass row of py (M[py % n][.]) given
// (loaded by the caller with its other global loads); same arithmetic.
template <typename T>
__device__ __forceinline__ Sides<T> zline_sides_row(const T (&row)[n], const T* ext, int N, const PatchPos& P,
                                                    int px, int py) {
  Sides<T> sd;
  sd.bl = (P.lo[2] == 0);
  sd.br = (P.lo[2] + 1 == N - 1);
  sd.aL = sd.bL = sd.aR = sd.bR = T(0);
  sd.lit = false;
  const int c0 = (py / n) * n;
  if (!sd.bl) {
    T s = T(0);
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += row[nu] * ext[px + E * (c0 + nu)];
    sd.bL = s;
  }
  if (!sd.br) {
    T s = T(0);
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += row[nu] * ext[NF + px + E * (c0 + nu)];
    sd.bR = s;
  }
  return sd;
}

// Read x-line (py, pz) from global.
template <typename T>
__device__ __forceinline__ void read_xline(const T* __restrict__ x, long long row0, Line<T>& v) {
#pragma unroll
  for (int a = 0; a < n; ++a) {
    v.v[a] = x[row0 + a];
    v.v[n + a] = x[row0 + NC + a];
  }
}

// Lines of a patch within one wave (3-D Q1, Q3: TPP = 16 or 64 lanes): values
// held one per lane can be contracted across lanes.
constexpr bool kZShfl = (TPP <= 64) && (64 % TPP == 0);

// sum_nu row[nu] v(lane + E (nu - mu)): the y-contraction of z-face values
// held one per lane (wl: the lane's index in its wave)
template <typename T>
__device__ __forceinline__ T ycontract_lanes(const T (&row)[n], T v, int wl, int mu) {
  T s = T(0);
#pragma unroll
  for (int nu = 0; nu < n; ++nu) s += row[nu] * __shfl(v, wl + E * (nu - mu), 64);
  return s;
}

// Couplings (alpha, beta) of one face node of a neighbour cell across a y-
// or z-face from the node's n values along the normal, v[j] (SIDE 0: the
// neighbour below, read at its far end; SIDE 1: above, read at its near end).
template <typename T, int SIDE>
__device__ __forceinline__ void face_node(T sg, const T (&v)[n], T& al, T& be) {
  const T half = T(0.5);
  T g = T(0), tr = T(0);
#pragma unroll
  for (int j = 0; j < n; ++j) {
    g += (SIDE == 0 ? T(kRef.d1[j]) : T(kRef.d0[j])) * v[j];
    if (j == (SIDE == 0 ? K : 0)) tr = v[j];
  }
  al = (SIDE == 0) ? (half * g - sg * tr) : (-sg * tr - half * g);
  be = (SIDE == 0) ? -half * tr : half * tr;
}

// Couplings of the n face nodes nu of an x-block of a neighbour cell across
// a y- or z-face; node nu, normal index j sits at c[nu + j strideN].
// a = sum_nu row[nu] alpha(nu), b = sum_nu row[nu] beta(nu).
template <typename T, int SIDE>
__device__ __forceinline__ void face_pair(const Tab<K, T>* __restrict__ t, const T* __restrict__ c,
                                          int strideN, const T (&row)[n], T& a, T& b) {
  const T sg = t->sigma;
  T al[n], be[n];
#pragma unroll
  for (int nu = 0; nu < n; ++nu) {
    T v[n];
#pragma unroll
    for (int j = 0; j < n; ++j) v[j] = c[nu + j * strideN];
    face_node<T, SIDE>(sg, v, al[nu], be[nu]);
  }
  T sa = T(0), sb = T(0);
#pragma unroll
  for (int nu = 0; nu < n; ++nu) sa += row[nu] * al[nu];
#pragma unroll
  for (int nu = 0; nu < n; ++nu) sb += row[nu] * be[nu];
  a = sa;
  b = sb;
}

// The lanes of an x-block (n consecutive lanes of a row of E) lie in one wave
// where E divides 64 (3-D Q1, Q3, Q7).
constexpr bool kXShfl = (64 % E) == 0;

// sum_nu row[nu] v(lane of node nu in this lane's x-block): the mass
// contraction of per-node face values held one per lane (wl: the lane's index
// in its wave, nuo: its node in the block); every lane of the block takes part
// Node NU of this lane's x-block, read by a DPP quad permutation (x-blocks of
// 2 or 4 lanes lie in one quad): a VALU move per 32 bits, no LDS crossbar.
template <int NU>
__device__ __forceinline__ constexpr int xblock_dpp() {
  return (n == 4) ? NU * 0x55 : (NU | (NU << 2) | ((2 + NU) << 4) | ((2 + NU) << 6));
}
template <int CTRL>
__device__ __forceinline__ double dpp_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <typename T>
__device__ __forceinline__ T xcontract_lanes(const T (&row)[n], T v, int wl, int nuo) {
  T s = T(0);
  if constexpr (n == 2 || n == 4) {
    s += row[0] * dpp_bcast<xblock_dpp<0>()>(v);
    s += row[1] * dpp_bcast<xblock_dpp<1>()>(v);
    if constexpr (n == 4) {
      s += row[2] * dpp_bcast<xblock_dpp<2>()>(v);
      s += row[3] * dpp_bcast<xblock_dpp<3>()>(v);
    }
  } else {
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += row[nu] * __shfl(v, wl - nuo + nu, 64);
  }
  return s;
}

// Dirichlet smoothers' z-face traces in registers (patches of one wave):
// lane (px, py) reads the n traces of its x-block on each z-neighbour and
// contracts beta = -+t/2 with its mass row (the values gather_ext +
// extz_mass_x_line leave in LDS) ...
template <typename T>
__device__ __forceinline__ void rfz_traces(const T* __restrict__ x, int N, const PatchPos& P, int lane,
                                           T& wz0, T& wz1) {
  const int px = lane % E, q = lane / E;
  T rowx[n];
  mass_row<T>(px % n, rowx);
  const T half = T(0.5);
  const int cx = P.lo[0] + px / n, cy = P.lo[1] + q / n;
  const long long o = (long long)n * (q % n);
  wz0 = wz1 = T(0);
  if (P.lo[2] > 0) {
    const T* c = x + cell_index(N, cx, cy, P.lo[2] - 1) * NC + o + K * n * n;
    T s = T(0);
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += rowx[nu] * (-half * c[nu]);
    wz0 = s;
  }
  if (P.lo[2] + 2 < N) {
    const T* c = x + cell_index(N, cx, cy, P.lo[2] + 2) * NC + o;
    T s = T(0);
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += rowx[nu] * (half * c[nu]);
    wz1 = s;
  }
}
// ... and the z-line (px, py = lane / E) contracts them along y across lanes
// (the values zline_sides forms from LDS); TRACES false: no neighbour data
template <typename T, bool TRACES>
__device__ __forceinline__ Sides<T> rfz_sides(int N, const PatchPos& P, int lane, T wz0, T wz1) {
  Sides<T> sd;
  sd.bl = (P.lo[2] == 0);
  sd.br = (P.lo[2] + 1 == N - 1);
  sd.aL = sd.bL = sd.aR = sd.bR = T(0);
  sd.lit = false;
  if constexpr (TRACES) {
    const int py = lane / E;
    T rowy[n];
    mass_row<T>(py % n, rowy);
    const int wl = threadIdx.x & 63;
    const T zL = ycontract_lanes<T>(rowy, wz0, wl, py % n);
    const T zR = ycontract_lanes<T>(rowy, wz1, wl, py % n);
    if (!sd.bl) sd.bL = zL;
    if (!sd.br) sd.bR = zR;
  }
  return sd;
}

// rfz_sides with traces, the mass row of py = lane / E given (loaded by the
// caller with its other global loads); same arithmetic
template <typename T>
__device__ __forceinline__ Sides<T> rfz_sides_row(const T (&rowy)[n], int N, const PatchPos& P, int lane, T wz0,
                                                  T wz1) {
  Sides<T> sd;
  sd.bl = (P.lo[2] == 0);
  sd.br = (P.lo[2] + 1 == N - 1);
  sd.aL = sd.bL = sd.aR = sd.bR = T(0);
  sd.lit = false;
  const int py = lane / E;
  const int wl = threadIdx.x & 63;
  const T zL = ycontract_lanes<T>(rowy, wz0, wl, py % n);
  const T zR = ycontract_lanes<T>(rowy, wz1, wl, py % n);
  if (!sd.bl) sd.bL = zL;
  if (!sd.br) sd.bR = zR;
  return sd;
}

// Operator passes of y = A_ref x on the patch.  Phase X0 reads the x-lines
// from global (and keeps them in xl for the caller), gathers the y/z face
// data; the last pass (z in 3-D, y in 2-D) hands each output line to
// emit(line, base, stride, y).  A, B: LDS tiles; ext: LDS face data.
// RFA (operator data, patches of one wave): the y- and z-neighbour face data
// in registers and across lanes as in k_apply_rf instead of the LDS arrays.
template <typename T, int MODE, bool RFA = false, typename Emit>
__device__ __forceinline__ void operator_passes(const Tab<K, T>* __restrict__ t, const T* __restrict__ x,
                                                int N, const PatchPos& P, T* A, T* B, T* ext,
                                                int lane, bool active, Line<T>& xl, Emit emit) {
  constexpr int NCOMP = (MODE == 0) ? 2 : 1;
  // Dirichlet smoothers on patches of one wave: the z-face traces go through
  // registers, not LDS.  Lane (px, py) reads the n traces of its x-block on
  // each z-neighbour and contracts beta = -+t/2 with its mass row (as
  // gather_ext + extz_mass_x_line), the Z pass contracts along y across lanes
  // (as ext_my): the same values, no extra pass over the face arrays.
  constexpr bool RFZ = (D == 3) && kZShfl && (MODE == 1 || MODE == 2);
  static_assert(!RFA || (MODE == 0 && D == 3 && kZShfl), "register face data: 3-D operator, one wave");
  T wz0 = T(0), wz1 = T(0);
  T ya0 = T(0), yb0 = T(0), ya1 = T(0), yb1 = T(0);  // RFA: y-line (px, pz) = (lane % E, lane / E)
  T za0 = T(0), zb0 = T(0), za1 = T(0), zb1 = T(0);  // RFA: z-face node (px, py) = (lane % E, lane / E)
  // the smoothers' residual is only used on V_j: along each direction the two
  // tile ends are skipped unless they lie on the domain boundary (outputs left
  // at the ends are never read by a used result)
  const bool n0x = MODE == 0 || (P.ty[0] & 1), nEx = MODE == 0 || (P.ty[0] & 2);
  const bool n0y = MODE == 0 || (P.ty[1] & 1), nEy = MODE == 0 || (P.ty[1] & 2);
  const bool n0z = MODE == 0 || (P.ty[2] & 1), nEz = MODE == 0 || (P.ty[2] & 2);
  // smoothers: y-face sides of the lane's y-line straight from global, and
  // (RFZ) the mass row of the z-line's py for the Z pass
  Sides<T> ysd_global{};
  T rowz[n];
  // X0: a = M_x x -> A, b = L_x x -> B
  if (active && MODE != 0 && NL == TPP) {
    // Smoothers with one line per lane: every global load of the pass is
    // issued before any of the values is used (one memory round trip instead
    // of one per helper), then the arithmetic of yline_sides_global,
    // rfz_traces and xline_sides in their order.
    const int px = lane % E, q = lane / E;  // y-line (px, pz = q), z-face node (px, py = q)
    YSideRaw<T> yraw;
    yside_load<T, MODE>(x, N, P, px, (D == 3) ? q : 0, yraw);
    T zl[n], zr[n];
    if constexpr (RFZ && MODE == 1) {
      const int cx = P.lo[0] + px / n, cy = P.lo[1] + q / n;
      const long long o = (long long)n * (q % n);
      const T* cl = x + cell_index(N, cx, cy, P.lo[2] > 0 ? P.lo[2] - 1 : P.lo[2]) * NC + o + K * n * n;
      const T* cr = x + cell_index(N, cx, cy, P.lo[2] + 2 < N ? P.lo[2] + 2 : P.lo[2]) * NC + o;
#pragma unroll
      for (int nu = 0; nu < n; ++nu) {
        zl[nu] = cl[nu];
        zr[nu] = cr[nu];
      }
      mass_row<T>(q % n, rowz);
    }
    // patches of several waves (no register z-faces): this lane's z-face node
    // (px, q) on both z-neighbours, the traces gather_ext would read
    T ztr0 = T(0), ztr1 = T(0);
    if constexpr (D == 3 && !RFZ && MODE == 1) {
      static_assert(NF == TPP, "one z-face node per lane");
      const int cx = P.lo[0] + px / n, cy = P.lo[1] + q / n;
      const long long o = px % n + (long long)n * (q % n);
      ztr0 = x[cell_index(N, cx, cy, P.lo[2] > 0 ? P.lo[2] - 1 : P.lo[2]) * NC + o + K * n * n];
      ztr1 = x[cell_index(N, cx, cy, P.lo[2] + 2 < N ? P.lo[2] + 2 : P.lo[2]) * NC + o];
    }
    const int py = lane % E, pz = lane / E;
    const long long row0 = xrow_offset(N, P, py, pz);
    read_xline<T>(x, row0, xl);
    const bool xbl = (P.lo[0] == 0), xbr = (P.lo[0] + 1 == N - 1);
    T xtl = T(0), xtr = T(0);
    if (MODE != 2) {
      xtl = x[xbl ? row0 : row0 - NC + K];
      xtr = x[xbr ? row0 : row0 + 2 * NC];
    }
    ysd_global = yside_finish<T, MODE>(yraw, N, P);
    if constexpr (RFZ && MODE == 1) {
      const T half = T(0.5);
      if (P.lo[2] > 0) {
        T s = T(0);
#pragma unroll
        for (int nu = 0; nu < n; ++nu) s += yraw.row[nu] * (-half * zl[nu]);
        wz0 = s;
      }
      if (P.lo[2] + 2 < N) {
        T s = T(0);
#pragma unroll
        for (int nu = 0; nu < n; ++nu) s += yraw.row[nu] * (half * zr[nu]);
        wz1 = s;
      }
    } else if constexpr (!RFZ && D == 3) {
      // the z-face traces as gather_ext stores them (zeros for MODE 2)
      const T half = T(0.5);
      ext[lane] = (MODE == 1 && P.lo[2] > 0) ? -half * ztr0 : T(0);
      ext[NF + lane] = (MODE == 1 && P.lo[2] + 2 < N) ? half * ztr1 : T(0);
    }
    Sides<T> sd;
    sd.bl = xbl;
    sd.br = xbr;
    sd.aL = sd.bL = sd.aR = sd.bR = T(0);
    sd.lit = (MODE == 2);
    if (MODE != 2) {
      if (!sd.bl) sd.bL = -T(0.5) * xtl;
      if (!sd.br) sd.bR = T(0.5) * xtr;
    }
    int base, stride;
    line_geom(0, lane, base, stride);
    Line<T> a, b;
    line_mass<T>(t, xl, a, n0x, nEx);
    line_sipg<T, false>(t, xl, sd, b, n0x, nEx);
    store_line(A, base, stride, a);
    store_line(B, base, stride, b);
  } else if (RFA && active) {
    static_assert(!RFA || kXShfl, "x-blocks within a wave");
    // register face data (operator, patches of one wave): every global load
    // first, as in k_apply_rf -- this lane's node column of each neighbour
    // face block, the x-line and its x-neighbours' rows -- then the per-node
    // face couplings, contracted with M_x across the lanes of the x-block
    const int px = lane % E, q = lane / E, nuo = px % n;
    const int wl = threadIdx.x & 63;
    const int cx = P.lo[0] + px / n;
    const bool ybl = (P.lo[1] == 0), ybr = (P.lo[1] + 1 == N - 1);
    const bool zbl = (P.lo[2] == 0), zbr = (P.lo[2] + 1 == N - 1);
    T fy0[n], fy1[n], fz0[n], fz1[n];
    {
      const int cz = P.lo[2] + q / n;
      const long long o = (long long)(n * n) * (q % n) + nuo;
      const T* c0 = x + cell_index(N, cx, ybl ? P.lo[1] : P.lo[1] - 1, cz) * NC + o;
      const T* c1 = x + cell_index(N, cx, ybr ? P.lo[1] + 1 : P.lo[1] + 2, cz) * NC + o;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        fy0[j] = c0[j * n];
        fy1[j] = c1[j * n];
      }
    }
    {
      const int cy = P.lo[1] + q / n;
      const long long o = (long long)n * (q % n) + nuo;
      const T* c0 = x + cell_index(N, cx, cy, zbl ? P.lo[2] : P.lo[2] - 1) * NC + o;
      const T* c1 = x + cell_index(N, cx, cy, zbr ? P.lo[2] + 1 : P.lo[2] + 2) * NC + o;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        fz0[j] = c0[j * n * n];
        fz1[j] = c1[j * n * n];
      }
    }
    const int py = lane % E, pz = lane / E;
    const long long row0 = xrow_offset(N, P, py, pz);
    read_xline<T>(x, row0, xl);
    const bool xbl = (P.lo[0] == 0), xbr = (P.lo[0] + 1 == N - 1);
    T rl[n], rr[n];
    {
      const T* r0 = x + (xbl ? row0 : row0 - NC);
      const T* r1 = x + (xbr ? row0 : row0 + 2 * NC);
#pragma unroll
      for (int j = 0; j < n; ++j) {
        rl[j] = r0[j];
        rr[j] = r1[j];
      }
    }
    T rowx[n];
    mass_row<T>(nuo, rowx);
    mass_row<T>(q % n, rowz);
    const T sg = t->sigma;
    T nya0, nyb0, nya1, nyb1, nza0, nzb0, nza1, nzb1;
    face_node<T, 0>(sg, fy0, nya0, nyb0);
    face_node<T, 1>(sg, fy1, nya1, nyb1);
    face_node<T, 0>(sg, fz0, nza0, nzb0);
    face_node<T, 1>(sg, fz1, nza1, nzb1);
    const Sides<T> sd = xsides_rows<T>(sg, xbl, xbr, rl, rr);
    int base, stride;
    line_geom(0, lane, base, stride);
    Line<T> a, b;
    line_mass<T>(t, xl, a, n0x, nEx);
    line_sipg<T, false>(t, xl, sd, b, n0x, nEx);
    store_line(A, base, stride, a);
    store_line(B, base, stride, b);
    const T sya0 = xcontract_lanes<T>(rowx, nya0, wl, nuo), syb0 = xcontract_lanes<T>(rowx, nyb0, wl, nuo);
    const T sya1 = xcontract_lanes<T>(rowx, nya1, wl, nuo), syb1 = xcontract_lanes<T>(rowx, nyb1, wl, nuo);
    const T sza0 = xcontract_lanes<T>(rowx, nza0, wl, nuo), szb0 = xcontract_lanes<T>(rowx, nzb0, wl, nuo);
    const T sza1 = xcontract_lanes<T>(rowx, nza1, wl, nuo), szb1 = xcontract_lanes<T>(rowx, nzb1, wl, nuo);
    if (!ybl) { ya0 = sya0; yb0 = syb0; }
    if (!ybr) { ya1 = sya1; yb1 = syb1; }
    if (!zbl) { za0 = sza0; zb0 = szb0; }
    if (!zbr) { za1 = sza1; zb1 = szb1; }
  } else if (active) {
    if constexpr (MODE != 0) ysd_global = yline_sides_global<T, MODE>(t, x, N, P, lane % E, lane / E);
    if constexpr (RFZ) {
      if constexpr (MODE == 1) rfz_traces<T>(x, N, P, lane, wz0, wz1);
    } else if constexpr (RFA) {
      const int px = lane % E, q = lane / E;
      T rowx[n];
      mass_row<T>(px % n, rowx);
      const int cx = P.lo[0] + px / n;
      const long long oy = (long long)(n * n) * (q % n), oz = (long long)n * (q % n);
      const int cz = P.lo[2] + q / n, cy = P.lo[1] + q / n;
      if (P.lo[1] > 0) face_pair<T, 0>(t, x + cell_index(N, cx, P.lo[1] - 1, cz) * NC + oy, n, rowx, ya0, yb0);
      if (P.lo[1] + 2 < N) face_pair<T, 1>(t, x + cell_index(N, cx, P.lo[1] + 2, cz) * NC + oy, n, rowx, ya1, yb1);
      if (P.lo[2] > 0) face_pair<T, 0>(t, x + cell_index(N, cx, cy, P.lo[2] - 1) * NC + oz, n * n, rowx, za0, zb0);
      if (P.lo[2] + 2 < N) face_pair<T, 1>(t, x + cell_index(N, cx, cy, P.lo[2] + 2) * NC + oz, n * n, rowx, za1, zb1);
    } else {
      gather_ext<T, MODE>(t, x, N, P, lane, ext);
    }
    for (int i = lane; i < NL; i += TPP) {
      const int py = i % E, pz = i / E;
      const long long row0 = xrow_offset(N, P, py, pz);
      read_xline<T>(x, row0, xl);
      const Sides<T> sd = xline_sides<T, MODE>(t, x, N, P, row0);
      int base, stride;
      line_geom(0, i, base, stride);
      Line<T> a, b;
      line_mass<T>(t, xl, a, n0x, nEx);
      line_sipg<T, false>(t, xl, sd, b, n0x, nEx);
      store_line(A, base, stride, a);
      store_line(B, base, stride, b);
    }
  }
  __syncthreads();
  if constexpr (D == 3) {
    // Y: c = M_y b + L_y a -> B, d = M_y a -> A; z-face data contracted along x
    if (active) {
      // one y-line per lane (NL = TPP), then, without register face data,
      // lanes 0 .. 2 NCOMP E - 1 contract one z-face row each along x (the
      // z-face arrays; the y-lines read only the y-face arrays of ext)
      {
        const int i = lane;
        {
          const int px = i % E, pz = i / E;
          int base, stride;
          line_geom(1, i, base, stride);
          Line<T> a, b, c, d;
          load_line(A, base, stride, a);
          load_line(B, base, stride, b);
          Sides<T> sd;
          if constexpr (RFA) {
            sd.bl = (P.lo[1] == 0);
            sd.br = (P.lo[1] + 1 == N - 1);
            sd.aL = ya0;
            sd.bL = yb0;
            sd.aR = ya1;
            sd.bR = yb1;
            sd.lit = false;
          } else {
            sd = (MODE == 0) ? yline_sides<T, NCOMP>(t, ext, N, P, px, pz) : ysd_global;
          }
          line_mass<T>(t, b, c, n0y, nEy);
          line_sipg<T, true>(t, a, sd, c, n0y, nEy);
          line_mass<T>(t, a, d, n0y, nEy);
          store_line(B, base, stride, c);
          store_line(A, base, stride, d);
        }
      }
      if constexpr (!(RFZ || RFA))
        if (lane < 2 * NCOMP * E) extz_mass_x_line<T, NCOMP>(t, ext, lane);
    }
    __syncthreads();
    // Z: y = M_z c + L_z d
    if (active) {
      for (int i = lane; i < NL; i += TPP) {
        const int px = i % E, py = i / E;
        int base, stride;
        line_geom(2, i, base, stride);
        Line<T> c, d, y;
        load_line(B, base, stride, c);
        load_line(A, base, stride, d);
        Sides<T> sd;
        if constexpr (RFZ && MODE == 1 && NL == TPP) {
          sd = rfz_sides_row<T>(rowz, N, P, i, wz0, wz1);
        } else if constexpr (RFZ) {
          sd = rfz_sides<T, MODE == 1>(N, P, i, wz0, wz1);
        } else if constexpr (RFA) {
          const int wl = threadIdx.x & 63;
          const T zaL = ycontract_lanes<T>(rowz, za0, wl, py % n);
          const T zbL = ycontract_lanes<T>(rowz, zb0, wl, py % n);
          const T zaR = ycontract_lanes<T>(rowz, za1, wl, py % n);
          const T zbR = ycontract_lanes<T>(rowz, zb1, wl, py % n);
          sd.bl = (P.lo[2] == 0);
          sd.br = (P.lo[2] + 1 == N - 1);
          sd.aL = sd.bl ? T(0) : zaL;
          sd.bL = sd.bl ? T(0) : zbL;
          sd.aR = sd.br ? T(0) : zaR;
          sd.bR = sd.br ? T(0) : zbR;
          sd.lit = false;
        } else {
          sd = zline_sides<T, NCOMP>(t, ext, N, P, px, py);
        }
        sd.lit = (MODE == 2);
        line_mass<T>(t, c, y, n0z, nEz);
        line_sipg<T, true>(t, d, sd, y, n0z, nEz);
        emit(i, base, stride, y);
      }
    }
  } else {
    // Y (2-D): y = M_y b + L_y a
    if (active) {
      for (int i = lane; i < NL; i += TPP) {
        const int px = i;
        int base, stride;
        line_geom(1, i, base, stride);
        Line<T> a, b, y;
        load_line(A, base, stride, a);
        load_line(B, base, stride, b);
        const Sides<T> sd = (MODE == 0) ? yline_sides<T, NCOMP>(t, ext, N, P, px, 0) : ysd_global;
        line_mass<T>(t, b, y, n0y, nEy);
        line_sipg<T, true>(t, a, sd, y, n0y, nEy);
        emit(i, base, stride, y);
      }
    }
  }
}

// Load the last-direction line of b (z-line in 3-D, y-line in 2-D) at line l.
template <typename T>
__device__ __forceinline__ void read_lastline(const T* __restrict__ b, int N, const PatchPos& P, int l,
                                              Line<T>& v) {
  if constexpr (D == 3) {
    const long long base = node_offset(N, P, l % E, l / E, 0);
    const long long cz = (long long)N * N * NC;  // next cell in z
#pragma unroll
    for (int p = 0; p < E; ++p) v.v[p] = b[base + (p / n) * cz + (p % n) * (n * n)];
  } else {
    const long long base = node_offset(N, P, l, 0, 0);
    const long long cy = (long long)N * NC;      // next cell in y
#pragma unroll
    for (int p = 0; p < E; ++p) v.v[p] = b[base + (p / n) * cy + (p % n) * n];
  }
}

template <int NB, int NEXTV>
struct Smem {
  static constexpr int per_patch = NB * TS + NEXTV;
};

// ---------------------------------------------------------------- apply
template <typename T, int PPB, bool RP = false>
__global__ void __launch_bounds__(TPP * PPB)
k_apply(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, const T* __restrict__ x,
        T* __restrict__ y, long long ndof) {
  constexpr int PP = Smem<2, (D - 1) * 2 * 2 * NF>::per_patch;
  __shared__ T smem[PPB * PP];
  const int slot = slot_of(), lane = threadIdx.x % TPP;
  int pid, rhs;
  slot_work<PPB, RP>(g, slot, pid, rhs);
  const bool active = pid < g.npatch;
  T* A = smem + slot * PP;
  T* B = A + TS;
  T* ext = B + TS;
  const long long roff = (long long)rhs * ndof;
  const T* xr = x + roff;
  T* yr = y + roff;
  const PatchPos P = patch_pos(g, active ? pid : 0);
  Line<T> xl;
  operator_passes<T, 0>(t, xr, g.N, P, A, B, ext, lane, active, xl,
                        [&](int, int base, int stride, const Line<T>& v) {
#pragma unroll
                          for (int p = 0; p < E; ++p) A[base + p * stride] = scale * v.v[p];
                        });
  __syncthreads();
  // X2: contiguous row stores
  if (active) {
    for (int i = lane; i < NL; i += TPP) {
      const int py = i % E, pz = i / E;
      int base, stride;
      line_geom(0, i, base, stride);
      const long long row0 = xrow_offset(g.N, P, py, pz);
#pragma unroll
      for (int a = 0; a < n; ++a) {
        yr[row0 + a] = A[base + a];
        yr[row0 + NC + a] = A[base + n + a];
      }
    }
  }
}

// ------------------------------------------- apply, face data in registers
// The face data of the y- and z-neighbours need not be gathered per face node
// into LDS.  Lane l forms, for its y-line (px, pz) and for the z-face node
// (px, py) of the same lane number, the couplings alpha, beta of the n face
// nodes of its x-block from the neighbour's lines along the face normal, and
// contracts them with the mass row of px in registers.  The z-face values are
// then contracted along y: where the lines of a patch sit in one wave (Q1,
// Q3: TPP = 16 or 64 lanes) with the lanes of the same px in the y-block
// (lane offsets E (nu - mu), cross-lane reads), otherwise through a small LDS
// array of the x-contracted values.  Every value is the expression of
// gather_ext / ext_mx / extz_mass_x_line / ext_my in the same order, so the
// result equals k_apply bit for bit.  LDS per patch: the two tiles (Q3 in
// FP64: 9 KB instead of 13 KB, 16 patches per CU instead of 12), plus
// 4 E^2 values elsewhere (Q7 in FP64: 78 KB instead of 86 KB, two patches per
// CU instead of one).
constexpr bool kApplyRF = (D == 3);
constexpr int kApplyRFPP = 2 * TS + (kZShfl ? 0 : 4 * NF);

template <typename T>
__device__ __forceinline__ void restrict_tail(const PatchGrid& g, const PatchPos& P, T* A, T* __restrict__ bc,
                                              long long ndof_c, int rhs, int lane, bool active);

// One patch of the register-face operator (pid, right-hand side rhs; lane =
// thread within the patch, A = its LDS, active: the patch takes part; xl
// returns the lane's x-line of x).  What follows the operator's last pass:
//   RF_APPLY: y = scale A x on the patch cells;
//   RF_RESTRICT: the residual restriction of k_restrict, bc = P^T (b - scale
//     A x) into the patch's coarse cell (y is bc there), with the same values
//     (the operator output and the P^T contractions in the same order);
//   RF_EMIT: emit(l, base, stride, v) with the operator output v of z-line l
//     (as operator_passes hands it to the Full smoother), nothing after it.
// All on the smaller LDS footprint of this kernel (two tiles, plus four
// z-face rows where patches span several waves).
constexpr int RF_APPLY = 0, RF_RESTRICT = 1, RF_EMIT = 2;
template <typename T, int OUT, typename Emit = int>
__device__ __forceinline__ void apply_rf_body(const Tab<K, T>* t, const PatchGrid& g, T scale, const T* x, T* y,
                                              const T* b, long long ndof, long long ndof_c, int pid, int lane,
                                              T* A, int rhs, bool active, Line<T>& xl, Emit emit = 0) {
  // cross-lane reads stay within a patch's lanes, which lie in one wave
  static_assert(kApplyRF, "3-D only");
  const int wl = threadIdx.x & 63;
  T* B = A + TS;
  const long long roff = (long long)rhs * ndof;
  const T* xr = x + roff;
  const int N = g.N;
  const PatchPos P = patch_pos(g, active ? pid : 0);
  // lane = px + E q: y-line (px, pz = q), z-face node (px, py = q)
  const int px = lane % E, q = lane / E;
  T rowx[n], rowy[n];
  mass_row<T>(px % n, rowx);
  mass_row<T>(q % n, rowy);
  const bool ybl = (P.lo[1] == 0), ybr = (P.lo[1] + 1 == N - 1);
  const bool zbl = (P.lo[2] == 0), zbr = (P.lo[2] + 1 == N - 1);
  T ya0 = T(0), yb0 = T(0), ya1 = T(0), yb1 = T(0);
  T za0 = T(0), zb0 = T(0), za1 = T(0), zb1 = T(0);
  // per-node face couplings of this lane's node nuo of its x-block
  T nya0 = T(0), nyb0 = T(0), nya1 = T(0), nyb1 = T(0);
  T nza0 = T(0), nzb0 = T(0), nza1 = T(0), nzb1 = T(0);
  const int nuo = px % n;
  if (!kXShfl && active) {
    // x-blocks straddle waves: each lane reads whole face blocks
    const int cx = P.lo[0] + px / n;
    {
      const int cz = P.lo[2] + q / n;
      const long long o = (long long)(n * n) * (q % n);
      if (!ybl) face_pair<T, 0>(t, xr + cell_index(N, cx, P.lo[1] - 1, cz) * NC + o, n, rowx, ya0, yb0);
      if (!ybr) face_pair<T, 1>(t, xr + cell_index(N, cx, P.lo[1] + 2, cz) * NC + o, n, rowx, ya1, yb1);
    }
    {
      const int cy = P.lo[1] + q / n;
      const long long o = (long long)n * (q % n);
      if (!zbl) face_pair<T, 0>(t, xr + cell_index(N, cx, cy, P.lo[2] - 1) * NC + o, n * n, rowx, za0, zb0);
      if (!zbr) face_pair<T, 1>(t, xr + cell_index(N, cx, cy, P.lo[2] + 2) * NC + o, n * n, rowx, za1, zb1);
    }
    const int py = lane % E, pz = lane / E;
    const long long row0 = xrow_offset(N, P, py, pz);
    read_xline<T>(xr, row0, xl);
    const Sides<T> sd = xline_sides<T, 0>(t, xr, N, P, row0);
    int base, stride;
    line_geom(0, lane, base, stride);
    Line<T> a, b;
    line_mass<T>(t, xl, a);
    line_sipg<T, false>(t, xl, sd, b);
    store_line(A, base, stride, a);
    store_line(B, base, stride, b);
  } else if (kXShfl && active) {
    // Every global load first (one memory round trip): this lane's node
    // column of each neighbour face block (n values along the normal), the
    // x-line and the rows of its x-neighbours; missing neighbours read the
    // patch's own cells, whose values go unused.
    const int cx = P.lo[0] + px / n;
    T fy0[n], fy1[n], fz0[n], fz1[n];
    {
      const int cz = P.lo[2] + q / n;
      const long long o = (long long)(n * n) * (q % n) + nuo;
      const T* c0 = xr + cell_index(N, cx, ybl ? P.lo[1] : P.lo[1] - 1, cz) * NC + o;
      const T* c1 = xr + cell_index(N, cx, ybr ? P.lo[1] + 1 : P.lo[1] + 2, cz) * NC + o;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        fy0[j] = c0[j * n];
        fy1[j] = c1[j * n];
      }
    }
    {
      const int cy = P.lo[1] + q / n;
      const long long o = (long long)n * (q % n) + nuo;
      const T* c0 = xr + cell_index(N, cx, cy, zbl ? P.lo[2] : P.lo[2] - 1) * NC + o;
      const T* c1 = xr + cell_index(N, cx, cy, zbr ? P.lo[2] + 1 : P.lo[2] + 2) * NC + o;
#pragma unroll
      for (int j = 0; j < n; ++j) {
        fz0[j] = c0[j * n * n];
        fz1[j] = c1[j * n * n];
      }
    }
    const int py = lane % E, pz = lane / E;
    const long long row0 = xrow_offset(N, P, py, pz);
    read_xline<T>(xr, row0, xl);
    const bool xbl = (P.lo[0] == 0), xbr = (P.lo[0] + 1 == N - 1);
    T rl[n], rr[n];
    {
      const T* r0 = xr + (xbl ? row0 : row0 - NC);
      const T* r1 = xr + (xbr ? row0 : row0 + 2 * NC);
#pragma unroll
      for (int j = 0; j < n; ++j) {
        rl[j] = r0[j];
        rr[j] = r1[j];
      }
    }
    const T sg = t->sigma;
    face_node<T, 0>(sg, fy0, nya0, nyb0);
    face_node<T, 1>(sg, fy1, nya1, nyb1);
    face_node<T, 0>(sg, fz0, nza0, nzb0);
    face_node<T, 1>(sg, fz1, nza1, nzb1);
    // X0: a = M_x x -> A, b = L_x x -> B
    const Sides<T> sd = xsides_rows<T>(sg, xbl, xbr, rl, rr);
    int base, stride;
    line_geom(0, lane, base, stride);
    Line<T> a, b;
    line_mass<T>(t, xl, a);
    line_sipg<T, false>(t, xl, sd, b);
    store_line(A, base, stride, a);
    store_line(B, base, stride, b);
  }
  // face couplings contracted with M_x across the lanes of each x-block
  // (all lanes of a patch take part)
  if constexpr (kXShfl) {
    const T sya0 = xcontract_lanes<T>(rowx, nya0, wl, nuo), syb0 = xcontract_lanes<T>(rowx, nyb0, wl, nuo);
    const T sya1 = xcontract_lanes<T>(rowx, nya1, wl, nuo), syb1 = xcontract_lanes<T>(rowx, nyb1, wl, nuo);
    const T sza0 = xcontract_lanes<T>(rowx, nza0, wl, nuo), szb0 = xcontract_lanes<T>(rowx, nzb0, wl, nuo);
    const T sza1 = xcontract_lanes<T>(rowx, nza1, wl, nuo), szb1 = xcontract_lanes<T>(rowx, nzb1, wl, nuo);
    if (!ybl) { ya0 = sya0; yb0 = syb0; }
    if (!ybr) { ya1 = sya1; yb1 = syb1; }
    if (!zbl) { za0 = sza0; zb0 = szb0; }
    if (!zbr) { za1 = sza1; zb1 = szb1; }
  }
  if constexpr (!kZShfl) {  // x-contracted z-face values for the y-contraction
    if (active) {
      T* wz = B + TS;
      wz[0 * NF + lane] = za0;
      wz[1 * NF + lane] = zb0;
      wz[2 * NF + lane] = za1;
      wz[3 * NF + lane] = zb1;
    }
  }
  __syncthreads();
  // Y: c = M_y b + L_y a -> B, d = M_y a -> A
  if (active) {
    int base, stride;
    line_geom(1, lane, base, stride);
    Line<T> a, b, c, d;
    load_line(A, base, stride, a);
    load_line(B, base, stride, b);
    Sides<T> sd;
    sd.bl = ybl;
    sd.br = ybr;
    sd.aL = ya0;
    sd.bL = yb0;
    sd.aR = ya1;
    sd.bR = yb1;
    sd.lit = false;
    line_mass<T>(t, b, c);
    line_sipg<T, true>(t, a, sd, c);
    line_mass<T>(t, a, d);
    store_line(B, base, stride, c);
    store_line(A, base, stride, d);
  }
  // z-face values contracted along y (all lanes of a patch take part)
  const int muy = q % n;
  T zaL = T(0), zbL = T(0), zaR = T(0), zbR = T(0);
  if constexpr (kZShfl) {
    zaL = ycontract_lanes<T>(rowy, za0, wl, muy);
    zbL = ycontract_lanes<T>(rowy, zb0, wl, muy);
    zaR = ycontract_lanes<T>(rowy, za1, wl, muy);
    zbR = ycontract_lanes<T>(rowy, zb1, wl, muy);
  }
  __syncthreads();
  if constexpr (!kZShfl) {
    if (active) {
      const T* wz = B + TS;
      const int f0 = px + E * (q - muy);
#pragma unroll
      for (int nu = 0; nu < n; ++nu) zaL += rowy[nu] * wz[0 * NF + f0 + E * nu];
#pragma unroll
      for (int nu = 0; nu < n; ++nu) zbL += rowy[nu] * wz[1 * NF + f0 + E * nu];
#pragma unroll
      for (int nu = 0; nu < n; ++nu) zaR += rowy[nu] * wz[2 * NF + f0 + E * nu];
#pragma unroll
      for (int nu = 0; nu < n; ++nu) zbR += rowy[nu] * wz[3 * NF + f0 + E * nu];
    }
  }
  // Z: y = M_z c + L_z d
  if (active) {
    int base, stride;
    line_geom(2, lane, base, stride);
    Line<T> c, d, o;
    load_line(B, base, stride, c);
    load_line(A, base, stride, d);
    Sides<T> sd;
    sd.bl = zbl;
    sd.br = zbr;
    sd.aL = zbl ? T(0) : zaL;
    sd.bL = zbl ? T(0) : zbL;
    sd.aR = zbr ? T(0) : zaR;
    sd.bR = zbr ? T(0) : zbR;
    sd.lit = false;
    line_mass<T>(t, c, o);
    line_sipg<T, true>(t, d, sd, o);
    if constexpr (OUT == RF_EMIT) {
      emit(lane, base, stride, o);
    } else if constexpr (OUT == RF_RESTRICT) {
      // r = b - scale A x on this z-line, contracted with P^T along z
      Line<T> r;
      read_lastline<T>(b + roff, N, P, lane, r);
#pragma unroll
      for (int nu = 0; nu < n; ++nu) {
        T s = T(0);
#pragma unroll
        for (int p = 0; p < E; ++p) s += T(kRef.P[p * n + nu]) * (r.v[p] - scale * o.v[p]);
        A[base + nu * stride] = s;
      }
    } else {
#pragma unroll
      for (int p = 0; p < E; ++p) A[base + p * stride] = scale * o.v[p];
    }
  }
  if constexpr (OUT == RF_EMIT) return;  // the caller's barrier follows
  __syncthreads();
  if constexpr (OUT == RF_RESTRICT) {
    restrict_tail<T>(g, P, A, y, ndof_c, rhs, lane, active);
  } else {
    // X2: contiguous row stores
    if (active) {
      T* yr = y + roff;
      const int py = lane % E, pz = lane / E;
      int base, stride;
      line_geom(0, lane, base, stride);
      const long long row0 = xrow_offset(N, P, py, pz);
#pragma unroll
      for (int a = 0; a < n; ++a) {
        yr[row0 + a] = A[base + a];
        yr[row0 + NC + a] = A[base + n + a];
      }
    }
  }
}

template <typename T, int PPB, bool RP = false>
__global__ void __launch_bounds__(TPP * PPB)
k_apply_rf(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, const T* __restrict__ x,
           T* __restrict__ y, long long ndof) {
  __shared__ T smem[PPB * kApplyRFPP];
  const int slot = slot_of(), lane = threadIdx.x % TPP;
  int pid, rhs;
  slot_work<PPB, RP>(g, slot, pid, rhs);
  Line<T> xl;
  apply_rf_body<T, RF_APPLY>(t, g, scale, x, y, nullptr, ndof, 0, pid, lane, smem + slot * kApplyRFPP, rhs,
                             pid < g.npatch, xl);
}

// ----------------------------------------------------------------- mass
template <typename T, int PPB>
__global__ void __launch_bounds__(TPP * PPB)
k_mass(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, const T* __restrict__ x,
       T* __restrict__ y, long long ndof) {
  __shared__ T smem[PPB * TS];
  const int slot = slot_of(), lane = threadIdx.x % TPP;
  const int pid = xcd_block(blockIdx.x, gridDim.x, g.xcd_remap) * PPB + slot;
  const bool active = pid < g.npatch;
  T* tile = smem + slot * TS;
  const long long roff = (long long)blockIdx.y * ndof;
  const PatchPos P = patch_pos(g, active ? pid : 0);
  if (active) {
    for (int i = lane; i < NL; i += TPP) {
      const int py = i % E, pz = i / E;
      int base, stride;
      line_geom(0, i, base, stride);
      Line<T> v, o;
      read_xline<T>(x + roff, xrow_offset(g.N, P, py, pz), v);
      line_mass<T>(t, v, o);
      store_line(tile, base, stride, o);
    }
  }
  __syncthreads();
#pragma unroll
  for (int dir = 1; dir < D; ++dir) {
    if (active) {
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(dir, i, base, stride);
        Line<T> v, o;
        load_line(tile, base, stride, v);
        line_mass<T>(t, v, o);
        store_line(tile, base, stride, o);
      }
    }
    __syncthreads();
  }
  if (active) {
    for (int i = lane; i < NL; i += TPP) {
      const int py = i % E, pz = i / E;
      int base, stride;
      line_geom(0, i, base, stride);
      const long long row0 = xrow_offset(g.N, P, py, pz);
#pragma unroll
      for (int a = 0; a < n; ++a) {
        y[roff + row0 + a] = scale * tile[base + a];
        y[roff + row0 + NC + a] = scale * tile[base + n + a];
      }
    }
  }
}

// -------------------------------------------------------------- smoother
// One colour of Alg. 1: local residual on the patch, then fast
// diagonalisation x|V_j += (x)S (sum lambda)^{-1} (x)S^T r_j.
//   MODE 1: Dirichlet kernel, consistent residual (b - A x)|V_j, in place;
//   MODE 2: Dirichlet kernel, the paper's residual: patch cells only, the
//           consistency term left out on interior outer faces; in place;
//   MODE 3: Full kernel: V_j = the whole patch, r = (b - A x)|patch with x taken
//           from xin, result written to xout.  Same-colour patches read each
//           other's cells (face neighbours), so the colour reads one copy of x
//           and writes the other; the launch also carries the partial patches
//           at the mesh boundary, which copy their in-domain cells unchanged.
//   MODE 4: clamped kernel: the residual from the patch cells alone (the
//           terms it misses act on directions the clamped space annihilates),
//           the FD solve on the clamped space; in place.
// ZERO: x = 0 on entry and the launch is colour 0, whose patches tile the mesh:
// the residual is b itself (no operator pass, x is not read) and every tile
// row is written (zeros outside V_j), so x needs no clearing beforehand.
// LDS per patch of the smoother: operator face data (full rows) for the Full
// kernel, z-face traces only for the Dirichlet and clamped kernels
// The Full kernel's operator pass takes the neighbour face data in registers
// in 3-D, as the apply and the restriction do: on patches within one wave (Q1,
// Q3) through operator_passes (two tiles of LDS per patch), otherwise through
// the apply's register-face body (two tiles and four z-face rows); no face
// arrays either way.
constexpr bool kFullRF = (D == 3) && kZShfl && kXShfl;
constexpr bool kFullOnApplyRF = kApplyRF && !kFullRF;
template <int MODE>
__host__ __device__ constexpr int smooth_pp() {
  return MODE == 3 ? (kFullRF ? 2 * TS : kFullOnApplyRF ? kApplyRFPP : Smem<2, (D - 1) * 2 * 2 * NF>::per_patch)
                   : Smem<2, (D - 2) * 2 * NF>::per_patch;
}

// One patch (pid of grid g, right-hand side rhs) of one colour; lane = thread
// within the patch, sm = the patch's LDS.  Every thread of the workgroup calls
// this (barriers inside), with pid >= g.npatch for idle slots.
template <typename T, int MODE, bool PREFETCH, bool ZERO>
__device__ __forceinline__ void smooth_body(const Tab<K, T>* __restrict__ t, const PatchGrid& g, T scale,
                                            T inv_scale, const T* __restrict__ xin, T* __restrict__ xout,
                                            const T* __restrict__ b, long long ndof, int pid, int lane,
                                            T* sm, int rhs) {
  constexpr bool FULL = (MODE == 3);
  constexpr int SP = FULL ? SP_FULL : (MODE == 4) ? SP_CLAMPED : SP_DIR;
  constexpr int OPM = FULL ? 0 : (MODE == 4) ? 2 : MODE;  // operator-pass mode (side data)
  const bool inrange = pid < g.npatch;
  T* A = sm;
  T* B = A + TS;
  T* ext = B + TS;
  const long long roff = (long long)rhs * ndof;
  T* xw = xout + roff;
  const T* xr = (FULL ? xin : xout) + roff;
  const T* br = b + roff;
  const PatchPos P = patch_pos(g, inrange ? pid : 0);
  bool whole = true;  // partial patches exist only in the Full kernel's launches
  if (FULL) {
#pragma unroll
    for (int i = 0; i < D; ++i) whole = whole && P.lo[i] >= 0 && P.lo[i] + 1 < g.N;
  }
  const bool active = inrange && whole;
  if (FULL && inrange && !whole) {
    // partial patch: copy the rows of its in-domain cells
    for (int i = lane; i < NL; i += TPP) {
      const int py = i % E, pz = i / E;
      const int cy = P.lo[1] + py / n;
      const int cz = (D == 3) ? P.lo[2] + pz / n : 0;
      if (cy < 0 || cy >= g.N || cz < 0 || cz >= g.N) continue;
      if (D == 2 && pz > 0) continue;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int cx = P.lo[0] + c;
        if (cx < 0 || cx >= g.N) continue;
        const long long row = cell_index(g.N, cx, cy, cz) * NC + (py % n) * n + ((D == 3) ? (pz % n) * n * n : 0);
#pragma unroll
        for (int a = 0; a < n; ++a) xw[row + a] = xr[row + a];
      }
    }
  }
  const int tyx = P.ty[0], tyy = P.ty[1], tyz = P.ty[2];
  // inverse eigenvalue sums of the lane's scaling line: read at the start in
  // 2-D (used by the first contraction phase), in 3-D only once the residual
  // is formed, so that they are not held through the operator passes (the
  // loads still overlap the X1 phase)
  T rsl[E];
  if (D == 2 && active) load_rs<T, SP>(t, P.ty, lane, rsl);
  Line<T> xl;  // the thread's x-line of x, kept for the final update
  // y-face couplings of the thread's y-line, read early from global (Dirichlet
  // kernels), and (PREFETCH) its line of b for the last operator pass: one
  // memory round trip less on the critical path of a patch, one tile more in
  // flight per patch
  if constexpr (ZERO) {
    // r = b, contracted with S^T along the last direction
#pragma unroll
    for (int p = 0; p < E; ++p) xl.v[p] = T(0);
    if (active)
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(D - 1, i, base, stride);
        Line<T> r, o;
        read_lastline<T>(br, g.N, P, i, r);
        line_St<T, SP>(t, (D == 3) ? tyz : tyy, r, o);
        store_line(A, base, stride, o);
      }
  } else {
    Line<T> bline;
    if (PREFETCH && active) read_lastline<T>(br, g.N, P, lane, bline);

    // residual r = b - A x on the last pass, contracted with S^T of that direction
    auto emit = [&](int l, int base, int stride, const Line<T>& v) {
      Line<T> r, o;
      if (PREFETCH) r = bline;
      else read_lastline<T>(br, g.N, P, l, r);
#pragma unroll
      for (int p = 0; p < E; ++p) r.v[p] -= scale * v.v[p];
      line_St<T, SP>(t, (D == 3) ? tyz : tyy, r, o);
      store_line(A, base, stride, o);
    };
    if constexpr (FULL && kFullOnApplyRF)
      apply_rf_body<T, RF_EMIT>(t, g, scale, xin, nullptr, nullptr, ndof, 0, pid, lane, A, rhs, active, xl, emit);
    else
      operator_passes<T, OPM, FULL && kFullRF>(t, xr, g.N, P, A, B, ext, lane, active, xl, emit);
  }
  __syncthreads();
  if constexpr (D == 3) {
    if (active) load_rs<T, SP>(t, P.ty, lane, rsl);
    // X1: S_x^T
    if (active)
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(0, i, base, stride);
        Line<T> v, o;
        load_line(A, base, stride, v);
        line_St<T, SP>(t, tyx, v, o);
        store_line(A, base, stride, o);
      }
    __syncthreads();
    // Y1: S_y^T, scale by 1/(sum lambda), S_y (one line per lane: TPP = NL)
    if (active)
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(1, i, base, stride);
        Line<T> v, o;
        load_line(A, base, stride, v);
        line_St<T, SP>(t, tyy, v, o);
#pragma unroll
        for (int q = 0; q < E; ++q) o.v[q] = o.v[q] * (inv_scale * rsl[q]);
        line_S<T, SP>(t, tyy, o, v);
        store_line(A, base, stride, v);
      }
    __syncthreads();
    // Z1: S_z
    if (active)
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(2, i, base, stride);
        Line<T> v, o;
        load_line(A, base, stride, v);
        line_S<T, SP>(t, tyz, v, o);
        store_line(A, base, stride, o);
      }
    __syncthreads();
  } else {
    // X1: S_x^T, scale, S_x (one line per lane: TPP = NL)
    if (active)
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(0, i, base, stride);
        Line<T> v, o;
        load_line(A, base, stride, v);
        line_St<T, SP>(t, tyx, v, o);
#pragma unroll
        for (int q = 0; q < E; ++q) o.v[q] = o.v[q] * (inv_scale * rsl[q]);
        line_S<T, SP>(t, tyx, o, v);
        store_line(A, base, stride, v);
      }
    __syncthreads();
    // Y1: S_y
    if (active)
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(1, i, base, stride);
        Line<T> v, o;
        load_line(A, base, stride, v);
        line_S<T, SP>(t, tyy, v, o);
        store_line(A, base, stride, o);
      }
    __syncthreads();
  }
  // X2 (3-D) / final x pass (2-D): x += S_x delta on the kept nodes, or, in
  // 3-D, x += delta with delta already in physical coordinates along x.
  if (active) {
    for (int i = lane; i < NL; i += TPP) {
      const int py = i % E, pz = i / E;
      const bool keep_line = FULL || ZERO ||
                             ((py > 0 || (tyy & 1)) && (py < E - 1 || (tyy & 2)) &&
                              (D == 2 || ((pz > 0 || (tyz & 1)) && (pz < E - 1 || (tyz & 2)))));
      if (!keep_line) continue;
      int base, stride;
      line_geom(0, i, base, stride);
      Line<T> dl;
      load_line(A, base, stride, dl);
      if constexpr (D == 3) {
        Line<T> o;
        line_S<T, SP>(t, tyx, dl, o);
        dl = o;
      }
      // whole rows: the dropped end nodes of a Dirichlet V_j are rewritten
      // with their unchanged value (delta is exactly zero there), so no
      // same-colour reader can observe a different value
      const long long row0 = xrow_offset(g.N, P, py, pz);
      Line<T> nx;
#pragma unroll
      for (int p = 0; p < E; ++p) nx.v[p] = xl.v[p] + dl.v[p];
      if (!FULL && !(tyx & 1)) nx.v[0] = xl.v[0];
      if (!FULL && !(tyx & 2)) nx.v[E - 1] = xl.v[E - 1];
#pragma unroll
      for (int a = 0; a < n; ++a) {
        xw[row0 + a] = nx.v[a];
        xw[row0 + NC + a] = nx.v[n + a];
      }
    }
  }
}

template <typename T, int PPB, int MODE, bool PREFETCH, bool ZERO = false, bool RP = false>
__global__ void __launch_bounds__(TPP * PPB)
k_smooth(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, T inv_scale,
         const T* __restrict__ xin, T* __restrict__ xout, const T* __restrict__ b, long long ndof) {
  constexpr int PP = smooth_pp<MODE>();
  __shared__ T smem[PPB * PP];
  const int slot = slot_of(), lane = threadIdx.x % TPP;
  int pid, rhs;
  slot_work<PPB, RP>(g, slot, pid, rhs);
  smooth_body<T, MODE, PREFETCH, ZERO>(t, g, scale, inv_scale, xin, xout, b, ndof, pid, lane,
                                       smem + slot * PP, rhs);
}


// ----------------------------------------------- split smoother (3-D)
// The same colour step with two waves per patch (TPP a multiple of 64): wave h
// of a patch owns, for every tile line, the outputs of cell h (indices
// h n .. h n + n - 1) -- or the eigen-coefficients q in that range in the
// fast-diagonalisation contractions -- while both waves read whole lines.
// The 1-D coefficients a wave needs stay wave-uniform, each output element is
// computed with the operations of the one-wave kernel in the same order (so
// the results are bitwise those of k_smooth), and a patch occupies twice the
// waves for the same LDS: more waves per SIMD to hide each other's latency.
// Phases that rewrite the tile they read put a barrier between the reads of
// both waves and the writes.
template <typename T>
struct Half {
  T v[n];
};

template <int H>
__device__ __forceinline__ constexpr bool half_end(int mu) { return H == 0 ? mu == 0 : mu == n - 1; }

// o = (blockdiag(M, M) v) on cell H; the patch-end output only if needEnd
template <typename T, int H>
__device__ __forceinline__ void half_mass(const Line<T>& v, Half<T>& o, bool needEnd) {
  if constexpr (kEOC) {
    T bl[n];
    cell_eo<T, true>(v, H, bl);
#pragma unroll
    for (int mu = 0; mu < n; ++mu) {
      if (half_end<H>(mu) && !needEnd) continue;
      o.v[mu] = bl[mu];
    }
    return;
  }
#pragma unroll
  for (int mu = 0; mu < n; ++mu) {
    if (half_end<H>(mu) && !needEnd) continue;
    T s = T(0);
#pragma unroll
    for (int nu = 0; nu < n; ++nu) s += T(kRef.M[mu * n + nu]) * v.v[H * n + nu];
    o.v[mu] = s;
  }
}

// o (+)= 1-D SIPG of the patch line v on cell H (the rows of line_sipg, in
// its order of operations)
template <typename T, int H, bool ACC>
__device__ __forceinline__ void half_sipg(const Tab<K, T>* __restrict__ t, const Line<T>& v,
                                          const Sides<T>& sd, Half<T>& o, bool needEnd) {
  const T sg = t->sigma;
  const T half = T(0.5);
  T bl[n];
  if constexpr (kEOC) cell_eo<T, false>(v, H, bl);
#pragma unroll
  for (int mu = 0; mu < n; ++mu) {
    if (half_end<H>(mu) && !needEnd) continue;
    T s = ACC ? o.v[mu] : T(0);
    if constexpr (kEOC) {
      s += bl[mu];
    } else {
#pragma unroll
      for (int nu = 0; nu < n; ++nu) s += T(kRef.Lcons[mu * n + nu]) * v.v[H * n + nu];
    }
    if (mu == 0) s += sg * v.v[H * n];
    if (mu == n - 1) s += sg * v.v[H * n + n - 1];
    o.v[mu] = s;
  }
  if constexpr (H == 0) {
    const T tR = v.v[n];
    T gR = T(0);
#pragma unroll
    for (int j = 0; j < n; ++j) gR += T(kRef.d0[j]) * v.v[n + j];
    T aL = sd.aL, bL = sd.bL;
    if (sd.bl) {
      T g0 = T(0);
#pragma unroll
      for (int j = 0; j < n; ++j) g0 += T(kRef.d0[j]) * v.v[j];
      aL = half * g0;
      bL = half * v.v[0];
    }
    if (!sd.bl && sd.lit) bL = -half * v.v[0];
    const T bLc = half * tR;
    if (needEnd) {
      o.v[0] += aL;
      o.v[0] += T(kRef.d0[0]) * bL + T(kRef.d1[0]) * bLc;
    }
    o.v[n - 1] += -sg * tR - half * gR;
#pragma unroll
    for (int mu = 1; mu < n; ++mu) o.v[mu] += T(kRef.d0[mu]) * bL + T(kRef.d1[mu]) * bLc;
  } else {
    const T tL = v.v[n - 1];
    T gL = T(0);
#pragma unroll
    for (int j = 0; j < n; ++j) gL += T(kRef.d1[j]) * v.v[j];
    T aR = sd.aR, bR = sd.bR;
    if (sd.br) {
      T g1 = T(0);
#pragma unroll
      for (int j = 0; j < n; ++j) g1 += T(kRef.d1[j]) * v.v[n + j];
      aR = -half * g1;
      bR = -half * v.v[E - 1];
    }
    if (!sd.br && sd.lit) bR = half * v.v[E - 1];
    const T bRc = -half * tL;
    o.v[0] += half * gL - sg * tL;
    if (needEnd) {
      o.v[n - 1] += aR;
      o.v[n - 1] += T(kRef.d0[n - 1]) * bRc + T(kRef.d1[n - 1]) * bR;
    }
#pragma unroll
    for (int mu = 0; mu < n - 1; ++mu) o.v[mu] += T(kRef.d0[mu]) * bRc + T(kRef.d1[mu]) * bR;
  }
}

// o[j] = sum_p S[p][q] v[p], q = H n + j (coefficients of line_St_t)
template <typename T, int TY, int SP, int H>
__device__ __forceinline__ void half_St_t(const Tab<K, T>* __restrict__ t, const Line<T>& v, Half<T>& o) {
  using B = FDB<SP, TY>;
  const T* S = fd_S<T, SP>(t, TY);
  if constexpr (kEO && SP == SP_DIR && TY == 0) {
    T vp[kEOH], vm[kEOH];
    eo_split<T>(v, vp, vm);
#pragma unroll
    for (int j = 0; j < n; ++j) {
      const int q = H * n + j;
      o.v[j] = (q < 2 * kEOH) ? eo_coef<T>(S, vp, vm, q) : T(0);
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < n; ++j) {
    const int q = H * n + j;
    T s = T(0);
    if (q < B::QN) {
#pragma unroll
      for (int p = B::PLO; p < B::PHI; ++p) s += S[p * E + q] * v.v[p];
    }
    o.v[j] = s;
  }
}
// o[j] = sum_q S[p][q] v[q], p = H n + j
template <typename T, int TY, int SP, int H>
__device__ __forceinline__ void half_S_t(const Tab<K, T>* __restrict__ t, const Line<T>& v, Half<T>& o) {
  using B = FDB<SP, TY>;
  const T* S = fd_S<T, SP>(t, TY);
  if constexpr (kEO && SP == SP_DIR && TY == 0) {
#pragma unroll
    for (int j = 0; j < n; ++j) {
      const int p = H * n + j;
      if (p == 0 || p == E - 1) {
        o.v[j] = T(0);
      } else {
        const int k = (p <= kEOH) ? p - 1 : E - 2 - p;
        T e, d;
        eo_pair<T>(S, v, k, e, d);
        o.v[j] = (p <= kEOH) ? e + d : e - d;
      }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < n; ++j) {
    const int p = H * n + j;
    T s = T(0);
    if (p >= B::PLO && p < B::PHI) {
#pragma unroll
      for (int q = 0; q < B::QN; ++q) s += S[p * E + q] * v.v[q];
    }
    o.v[j] = s;
  }
}
template <typename T, int SP, int H>
__device__ __forceinline__ void half_St(const Tab<K, T>* __restrict__ t, int ty, const Line<T>& v, Half<T>& o) {
  switch (ty) {
    case 0: half_St_t<T, 0, SP, H>(t, v, o); break;
    case 1: half_St_t<T, 1, SP, H>(t, v, o); break;
    case 2: half_St_t<T, 2, SP, H>(t, v, o); break;
    default: half_St_t<T, 3, SP, H>(t, v, o); break;
  }
}
template <typename T, int SP, int H>
__device__ __forceinline__ void half_S(const Tab<K, T>* __restrict__ t, int ty, const Line<T>& v, Half<T>& o) {
  switch (ty) {
    case 0: half_S_t<T, 0, SP, H>(t, v, o); break;
    case 1: half_S_t<T, 1, SP, H>(t, v, o); break;
    case 2: half_S_t<T, 2, SP, H>(t, v, o); break;
    default: half_S_t<T, 3, SP, H>(t, v, o); break;
  }
}

template <typename T>
__device__ __forceinline__ void store_half(T* s, int base, int stride, int H, const Half<T>& o) {
#pragma unroll
  for (int j = 0; j < n; ++j) s[base + (H * n + j) * stride] = o.v[j];
}

// last-direction (z) line of b, the cells of half H only
template <typename T>
__device__ __forceinline__ void read_lasthalf(const T* __restrict__ b, int N, const PatchPos& P, int l, int H,
                                              Half<T>& v) {
  const long long base = node_offset(N, P, l % E, l / E, 0) + (long long)H * N * N * NC;
#pragma unroll
  for (int j = 0; j < n; ++j) v.v[j] = b[base + j * (n * n)];
}

constexpr bool kSplitOK = (D == 3) && (TPP % 64 == 0);

template <typename T, int MODE, bool PREFETCH, bool ZERO, int H>
__device__ __forceinline__ void smooth_split_body(const Tab<K, T>* __restrict__ t, const PatchGrid& g,
                                                  T scale, T inv_scale, T* __restrict__ x,
                                                  const T* __restrict__ b, long long ndof, int pid,
                                                  int lane, T* sm, int rhs) {
  static_assert(MODE != 3, "the Full kernel is not split");
  constexpr int SP = (MODE == 4) ? SP_CLAMPED : SP_DIR;
  constexpr int OPM = (MODE == 4) ? 2 : MODE;
  const bool active = pid < g.npatch;
  T* A = sm;
  T* B = A + TS;
  T* ext = B + TS;
  const long long roff = (long long)rhs * ndof;
  T* xr = x + roff;
  const T* br = b + roff;
  const PatchPos P = patch_pos(g, active ? pid : 0);
  const int tyx = P.ty[0], tyy = P.ty[1], tyz = P.ty[2];
  // ends of this half's cell that lie on the patch boundary are needed only
  // on the domain boundary (Dirichlet and clamped spaces)
  const bool endx = (tyx & (H == 0 ? 1 : 2)) != 0;
  const bool endy = (tyy & (H == 0 ? 1 : 2)) != 0;
  const bool endz = (tyz & (H == 0 ? 1 : 2)) != 0;
  Half<T> xh;  // this half of the thread's x-line of x
  Half<T> bh;  // this half of the thread's z-line of b
  T rsh[n];    // inverse eigenvalue sums of this half of the lane's scaling line
  if (PREFETCH && active) read_lasthalf<T>(br, g.N, P, lane, H, bh);
  if constexpr (ZERO) {
#pragma unroll
    for (int j = 0; j < n; ++j) xh.v[j] = T(0);
    if (active) {
      // r = b: this half to A, then S_z^T over whole lines into B
      if (!PREFETCH) read_lasthalf<T>(br, g.N, P, lane, H, bh);
      int base, stride;
      line_geom(2, lane, base, stride);
      store_half(A, base, stride, H, bh);
    }
    __syncthreads();
  } else {
    // Q3: every global load of the first phases is issued here, before any
    // of the values is used (one memory round trip instead of one per
    // helper): the y-neighbour traces with their mass row, this lane's z-face
    // trace, the x-line with its x-neighbour traces and the mass row of the
    // z-sides.  For 16-point lines the registers this holds would cost a
    // wave per SIMD, so there the helpers load one after the other.
    static_assert(TPP == NF, "one z-face trace per lane of the two waves");
    constexpr bool HOIST = (n <= 4);
    Sides<T> ysd{}, sd{};
    T zrow[n];
    Line<T> xl;
    const int py = lane % E, pz = lane / E;
    const long long row0 = xrow_offset(g.N, P, py, pz);
    if constexpr (HOIST) {
      YSideRaw<T> yraw;
      T ztr = T(0), xtl = T(0), xtr = T(0);
      const int zf = lane, zside = H;  // this lane's z-face entry (face node, side)
      const int znb = (zside == 0) ? P.lo[2] - 1 : P.lo[2] + 2;
      const bool zhas = MODE == 1 && znb >= 0 && znb < g.N;
      const bool xbl = (P.lo[0] == 0), xbr = (P.lo[0] + 1 == g.N - 1);
      if (active) {
        yside_load<T, OPM>(xr, g.N, P, lane % E, lane / E, yraw);
        if (MODE == 1) {
          const int a = zf % E, bb = zf / E;
          const long long base = cell_index(g.N, P.lo[0] + a / n, P.lo[1] + bb / n, zhas ? znb : P.lo[2]) * NC +
                                 a % n + n * (bb % n);
          ztr = xr[base + (long long)((zside == 0) ? K : 0) * n * n];
        }
        read_xline<T>(xr, row0, xl);
        if (OPM != 2) {
          xtl = xr[xbl ? row0 : row0 - NC + K];
          xtr = xr[xbr ? row0 : row0 + 2 * NC];
        }
        mass_row<T>((lane / E) % n, zrow);
        ysd = yside_finish<T, OPM>(yraw, g.N, P);
        // z-face traces, spread over both waves (the register form of the
        // one-wave kernel measured slower here: both waves would repeat it)
        ext[zside * NF + zf] = zhas ? ((zside == 0) ? -T(0.5) * ztr : T(0.5) * ztr) : T(0);
        // x-sides as xline_sides forms them for the smoother's residual
        sd.bl = xbl;
        sd.br = xbr;
        sd.aL = sd.bL = sd.aR = sd.bR = T(0);
        sd.lit = (OPM == 2);
        if (OPM != 2) {
          if (!sd.bl) sd.bL = -T(0.5) * xtl;
          if (!sd.br) sd.bR = T(0.5) * xtr;
        }
      }
    } else {
      // this lane's z-face entry (face node lane, side H), its load issued
      // before the y-side loads so that both arrive in one round trip
      const int znb = (H == 0) ? P.lo[2] - 1 : P.lo[2] + 2;
      const bool zhas = MODE == 1 && znb >= 0 && znb < g.N;
      T ztr = T(0);
      if (active && MODE == 1) {
        const int a = lane % E, bb = lane / E;
        const long long base = cell_index(g.N, P.lo[0] + a / n, P.lo[1] + bb / n, zhas ? znb : P.lo[2]) * NC +
                               a % n + n * (bb % n);
        ztr = xr[base + (long long)((H == 0) ? K : 0) * n * n];
      }
      if (active) ysd = yline_sides_global<T, OPM>(t, xr, g.N, P, lane % E, lane / E);
      if (active) {
        ext[H * NF + lane] = zhas ? ((H == 0) ? -T(0.5) * ztr : T(0.5) * ztr) : T(0);
        read_xline<T>(xr, row0, xl);
        sd = xline_sides<T, OPM>(t, xr, g.N, P, row0);
      }
    }
    // X0: a = M_x x, b = L_x x on this half -> A, B
    if (active) {
#pragma unroll
      for (int j = 0; j < n; ++j) xh.v[j] = xl.v[H * n + j];
      int base, stride;
      line_geom(0, lane, base, stride);
      Half<T> a, bb;
      half_mass<T, H>(xl, a, endx);
      half_sipg<T, H, false>(t, xl, sd, bb, endx);
      store_half(A, base, stride, H, a);
      store_half(B, base, stride, H, bb);
    }
    __syncthreads();
    // Y: c = M_y b + L_y a -> B, d = M_y a -> A (after both waves have read)
    Half<T> c, d;
    int ybase = 0, ystride = 0;
    if (active) {
      const int px = lane % E, pz = lane / E;
      line_geom(1, lane, ybase, ystride);
      Line<T> a, bl;
      load_line(A, ybase, ystride, a);
      load_line(B, ybase, ystride, bl);
      (void)px;
      (void)pz;
      half_mass<T, H>(bl, c, endy);
      half_sipg<T, H, true>(t, a, ysd, c, endy);
      half_mass<T, H>(a, d, endy);
      // z-face traces contracted along x (16 rows, one per thread of wave 1)
      if (H == 1 && lane < 2 * E) extz_mass_x_line<T, 1>(t, ext, lane);
    }
    __syncthreads();
    if (active) {
      store_half(B, ybase, ystride, H, c);
      store_half(A, ybase, ystride, H, d);
    }
    __syncthreads();
    // Z: y = M_z c + L_z d, r = b - scale y on this half -> A, then S_z^T
    if (active) {
      const int px = lane % E, py = lane / E;
      int base, stride;
      line_geom(2, lane, base, stride);
      Line<T> cl, dl;
      load_line(B, base, stride, cl);
      load_line(A, base, stride, dl);
      Sides<T> sd;
      if constexpr (HOIST) sd = zline_sides_row<T>(zrow, ext, g.N, P, px, py);
      else sd = zline_sides<T, 1>(t, ext, g.N, P, px, py);
      sd.lit = (OPM == 2);
      Half<T> y;
      half_mass<T, H>(cl, y, endz);
      half_sipg<T, H, true>(t, dl, sd, y, endz);
      if (!PREFETCH) read_lasthalf<T>(br, g.N, P, lane, H, bh);
#pragma unroll
      for (int j = 0; j < n; ++j) bh.v[j] -= scale * y.v[j];
    }
    __syncthreads();
    if (active) {
      int base, stride;
      line_geom(2, lane, base, stride);
      store_half(A, base, stride, H, bh);
    }
    __syncthreads();
  }
  // (the eigenvalue sums are read only now, not held through the residual
  // passes; their loads overlap the next two phases)
  if (active) {
    T rsl[E];
    load_rs<T, SP>(t, P.ty, lane, rsl);
#pragma unroll
    for (int j = 0; j < n; ++j) rsh[j] = rsl[H * n + j];
  }
  // S_z^T over the whole residual line -> B
  if (active) {
    int base, stride;
    line_geom(2, lane, base, stride);
    Line<T> r;
    load_line(A, base, stride, r);
    Half<T> o;
    half_St<T, SP, H>(t, tyz, r, o);
    store_half(B, base, stride, H, o);
  }
  __syncthreads();
  // X1: S_x^T, B -> A
  if (active) {
    int base, stride;
    line_geom(0, lane, base, stride);
    Line<T> v;
    load_line(B, base, stride, v);
    Half<T> o;
    half_St<T, SP, H>(t, tyx, v, o);
    store_half(A, base, stride, H, o);
  }
  __syncthreads();
  // Y1a: S_y^T and 1/(sum lambda), A -> B
  if (active) {
    int base, stride;
    line_geom(1, lane, base, stride);
    Line<T> v;
    load_line(A, base, stride, v);
    Half<T> o;
    half_St<T, SP, H>(t, tyy, v, o);
#pragma unroll
    for (int j = 0; j < n; ++j) o.v[j] = o.v[j] * (inv_scale * rsh[j]);
    store_half(B, base, stride, H, o);
  }
  __syncthreads();
  // Y1b: S_y, B -> A
  if (active) {
    int base, stride;
    line_geom(1, lane, base, stride);
    Line<T> v;
    load_line(B, base, stride, v);
    Half<T> o;
    half_S<T, SP, H>(t, tyy, v, o);
    store_half(A, base, stride, H, o);
  }
  __syncthreads();
  // Z1: S_z, A -> B
  if (active) {
    int base, stride;
    line_geom(2, lane, base, stride);
    Line<T> v;
    load_line(A, base, stride, v);
    Half<T> o;
    half_S<T, SP, H>(t, tyz, v, o);
    store_half(B, base, stride, H, o);
  }
  __syncthreads();
  // X2: x += S_x delta on this half's cell row of the kept lines
  if (active) {
    const int py = lane % E, pz = lane / E;
    const bool keep_line = ZERO || ((py > 0 || (tyy & 1)) && (py < E - 1 || (tyy & 2)) &&
                                    (pz > 0 || (tyz & 1)) && (pz < E - 1 || (tyz & 2)));
    if (keep_line) {
      int base, stride;
      line_geom(0, lane, base, stride);
      Line<T> v;
      load_line(B, base, stride, v);
      Half<T> dl;
      half_S<T, SP, H>(t, tyx, v, dl);
      Half<T> nx;
#pragma unroll
      for (int j = 0; j < n; ++j) nx.v[j] = xh.v[j] + dl.v[j];
      if (H == 0 && !(tyx & 1)) nx.v[0] = xh.v[0];
      if (H == 1 && !(tyx & 2)) nx.v[n - 1] = xh.v[n - 1];
      const long long row = xrow_offset(g.N, P, py, pz) + (long long)H * NC;
#pragma unroll
      for (int j = 0; j < n; ++j) xr[row + j] = nx.v[j];
    }
  }
}

template <typename T, int PPB, int MODE, bool PREFETCH, bool ZERO = false>
__global__ void __launch_bounds__(2 * TPP * PPB)
k_smooth_split(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, T inv_scale, T* __restrict__ x,
               const T* __restrict__ b, long long ndof) {
  constexpr int PP = smooth_pp<1>();
  __shared__ T smem[PPB * PP];
  const int w = (int)threadIdx.x / TPP;  // wave group: slot * 2 + half
  const int ws = kSplitOK ? __builtin_amdgcn_readfirstlane(w) : w;
  const int slot = ws / 2, h = ws % 2, lane = threadIdx.x % TPP;
  const int pid = xcd_block(blockIdx.x, gridDim.x, g.xcd_remap) * PPB + slot;
  if (h == 0)
    smooth_split_body<T, MODE, PREFETCH, ZERO, 0>(t, g, scale, inv_scale, x, b, ndof, pid, lane,
                                                  smem + slot * PP, blockIdx.y);
  else
    smooth_split_body<T, MODE, PREFETCH, ZERO, 1>(t, g, scale, inv_scale, x, b, ndof, pid, lane,
                                                  smem + slot * PP, blockIdx.y);
}

// ------------------------------------------------- residual + restriction
// bc = P^T (b - A x): the colour-0 patch of level l is the set of children of
// one coarse cell, so its residual contracts with the stacked P^T per
// direction straight into that coarse cell.
// Q1, Q3 in 3-D: the operator pass takes the neighbour face data in registers
// (as the apply's shape 2): two tiles of LDS per patch, no face arrays.
constexpr bool kRestrictRF = (D == 3) && kZShfl;
constexpr int kRestrictPP = kRestrictRF ? 2 * TS : Smem<2, (D - 1) * 2 * 2 * NF>::per_patch;

template <typename T>
__device__ __forceinline__ void restrict_body(const Tab<K, T>* __restrict__ t, const PatchGrid& g, T scale,
                                              const T* __restrict__ x, const T* __restrict__ b,
                                              T* __restrict__ bc, long long ndof, long long ndof_c,
                                              int pid, int lane, T* sm, int rhs) {
  const bool active = pid < g.npatch;
  T* A = sm;
  T* B = A + TS;
  T* ext = B + TS;
  const long long roff = (long long)rhs * ndof;
  const PatchPos P = patch_pos(g, active ? pid : 0);
  Line<T> xl;
  operator_passes<T, 0, kRestrictRF>(t, x + roff, g.N, P, A, B, ext, lane, active, xl,
                        [&](int l, int base, int stride, const Line<T>& v) {
                          Line<T> r;
                          read_lastline<T>(b + roff, g.N, P, l, r);
#pragma unroll
                          for (int nu = 0; nu < n; ++nu) {
                            T s = T(0);
#pragma unroll
                            for (int p = 0; p < E; ++p) s += T(kRef.P[p * n + nu]) * (r.v[p] - scale * v.v[p]);
                            A[base + nu * stride] = s;
                          }
                        });
  __syncthreads();
  restrict_tail<T>(g, P, A, bc, ndof_c, rhs, lane, active);
}

// The restriction after the last direction (its P^T values at the first n
// nodes of each last-direction line of A): P^T along y (3-D), then along x
// into the rows of the patch's coarse cell of bc.
template <typename T>
__device__ __forceinline__ void restrict_tail(const PatchGrid& g, const PatchPos& P, T* A, T* __restrict__ bc,
                                              long long ndof_c, int rhs, int lane, bool active) {
  if constexpr (D == 3) {
    // restrict along y: lines (px, pz < n)
    if (active)
      for (int i = lane; i < E * n; i += TPP) {
        const int px = i % E, pz = i / E;
        const int base = px + pz * SZ, stride = SY;
        Line<T> v;
        load_line(A, base, stride, v);
#pragma unroll
        for (int nu = 0; nu < n; ++nu) {
          T s = T(0);
#pragma unroll
          for (int p = 0; p < E; ++p) s += T(kRef.P[p * n + nu]) * v.v[p];
          A[base + nu * stride] = s;
        }
      }
    __syncthreads();
  }
  // restrict along x: lines (py < n, pz < n) into rows of the coarse cell
  if (active) {
    const int Nc = g.N / 2;
    const long long cell = cell_index(Nc, P.lo[0] / 2, P.lo[1] / 2, (D == 3) ? P.lo[2] / 2 : 0);
    T* out = bc + (long long)rhs * ndof_c + cell * NC;
    for (int i = lane; i < NC / n; i += TPP) {
      const int py = i % n, pz = i / n;
      const int base = py * SY + pz * SZ;
      Line<T> v;
      load_line(A, base, 1, v);
#pragma unroll
      for (int nu = 0; nu < n; ++nu) {
        T s = T(0);
#pragma unroll
        for (int p = 0; p < E; ++p) s += T(kRef.P[p * n + nu]) * v.v[p];
        out[i * n + nu] = s;
      }
    }
  }
}

template <typename T, int PPB>
__global__ void __launch_bounds__(TPP * PPB)
k_restrict(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, const T* __restrict__ x,
           const T* __restrict__ b, T* __restrict__ bc, long long ndof, long long ndof_c) {
  __shared__ T smem[PPB * kRestrictPP];
  const int slot = slot_of(), lane = threadIdx.x % TPP;
  const int pid = xcd_block(blockIdx.x, gridDim.x, g.xcd_remap) * PPB + slot;
  restrict_body<T>(t, g, scale, x, b, bc, ndof, ndof_c, pid, lane, smem + slot * kRestrictPP, blockIdx.y);
}

// 3-D degrees whose patches span several waves (or do not divide one): the
// same restriction on the register-face operator of k_apply_rf, whose LDS
// holds two tiles and four z-face rows instead of the face arrays (3-D Q7 in
// FP64: two patches per CU instead of one)
constexpr bool kRestrictOnApplyRF = kApplyRF && !kRestrictRF;
template <typename T, int PPB>
__global__ void __launch_bounds__(TPP * PPB)
k_restrict_rf(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, const T* __restrict__ x,
              const T* __restrict__ b, T* __restrict__ bc, long long ndof, long long ndof_c) {
  __shared__ T smem[PPB * kApplyRFPP];
  const int slot = slot_of(), lane = threadIdx.x % TPP;
  const int pid = xcd_block(blockIdx.x, gridDim.x, g.xcd_remap) * PPB + slot;
  Line<T> xl;
  apply_rf_body<T, RF_RESTRICT>(t, g, scale, x, bc, b, ndof, ndof_c, pid, lane, smem + slot * kApplyRFPP,
                                blockIdx.y, pid < g.npatch, xl);
}

// ------------------------------------------------- prolongation + add
template <typename T>
__device__ __forceinline__ void prolong_body(const PatchGrid& g, const T* __restrict__ xc, T* __restrict__ x,
                                             long long ndof, long long ndof_c, int pid, int lane, T* tile,
                                             int rhs) {
  const bool active = pid < g.npatch;
  const PatchPos P = patch_pos(g, active ? pid : 0);
  const long long roff = (long long)rhs * ndof;
  // along x: coarse rows (ly, lz) straight from global
  if (active) {
    const int Nc = g.N / 2;
    const long long cell = cell_index(Nc, P.lo[0] / 2, P.lo[1] / 2, (D == 3) ? P.lo[2] / 2 : 0);
    const T* in = xc + (long long)rhs * ndof_c + cell * NC;
    for (int i = lane; i < NC / n; i += TPP) {
      const int py = i % n, pz = i / n;
      const int base = py * SY + pz * SZ;
      T v[n];
#pragma unroll
      for (int nu = 0; nu < n; ++nu) v[nu] = in[i * n + nu];
#pragma unroll
      for (int p = 0; p < E; ++p) {
        T s = T(0);
#pragma unroll
        for (int nu = 0; nu < n; ++nu) s += T(kRef.P[p * n + nu]) * v[nu];
        tile[base + p] = s;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int dir = 1; dir < D; ++dir) {
    if (active) {
      // lines along dir; coordinates in later directions still < n
      const int nlines = (D == 3 && dir == 1) ? E * n : E * E;
      for (int i = lane; i < (D == 2 ? E : nlines); i += TPP) {
        int base, stride;
        if (D == 3 && dir == 1) { const int px = i % E, pz = i / E; base = px + pz * SZ; stride = SY; }
        else line_geom(dir, i, base, stride);
        T v[n];
#pragma unroll
        for (int nu = 0; nu < n; ++nu) v[nu] = tile[base + nu * stride];
#pragma unroll
        for (int p = 0; p < E; ++p) {
          T s = T(0);
#pragma unroll
          for (int nu = 0; nu < n; ++nu) s += T(kRef.P[p * n + nu]) * v[nu];
          tile[base + p * stride] = s;
        }
      }
    }
    __syncthreads();
  }
  if (active) {
    for (int i = lane; i < NL; i += TPP) {
      const int py = i % E, pz = i / E;
      int base, stride;
      line_geom(0, i, base, stride);
      const long long row0 = roff + xrow_offset(g.N, P, py, pz);
#pragma unroll
      for (int a = 0; a < n; ++a) {
        x[row0 + a] += tile[base + a];
        x[row0 + NC + a] += tile[base + n + a];
      }
    }
  }
}

template <typename T, int PPB>
__global__ void __launch_bounds__(TPP * PPB)
k_prolong(const Tab<K, T>* __restrict__ t, PatchGrid g, const T* __restrict__ xc,
          T* __restrict__ x, long long ndof, long long ndof_c) {
  __shared__ T smem[PPB * TS];
  const int slot = slot_of(), lane = threadIdx.x % TPP;
  const int pid = xcd_block(blockIdx.x, gridDim.x, g.xcd_remap) * PPB + slot;
  (void)t;
  prolong_body<T>(g, xc, x, ndof, ndof_c, pid, lane, smem + slot * TS, blockIdx.y);
}

// ---------------------------------------------------------- coarse solve
// Level 0 (N = 2): one patch, every node kept (type 3 in all directions).
// Every thread of the workgroup calls this (barriers inside); only threads
// with active set work.
template <typename T>
__device__ __forceinline__ void coarse_body(const Tab<K, T>* __restrict__ t, T inv_scale,
                                            const T* __restrict__ b, T* __restrict__ x, long long ndof,
                                            int lane, T* tile, int rhs, bool active) {
  PatchPos P;
#pragma unroll
  for (int i = 0; i < 3; ++i) { P.lo[i] = 0; P.ty[i] = 3; }
  const long long roff = (long long)rhs * ndof;
  const int nl = active ? NL : 0;  // lines this thread's patch slot works on
  // S_x^T straight from the rows of b
  for (int i = lane; i < nl; i += TPP) {
    const int py = i % E, pz = i / E;
    int base, stride;
    line_geom(0, i, base, stride);
    Line<T> v, o;
    read_xline<T>(b + roff, xrow_offset(2, P, py, pz), v);
    line_St_t<T, 3, SP_DIR>(t, v, o);
    store_line(tile, base, stride, o);
  }
  __syncthreads();
  // S^T along the remaining directions; the last one also scales and applies S
#pragma unroll
  for (int dir = 1; dir < D; ++dir) {
    for (int i = lane; i < nl; i += TPP) {
      int base, stride;
      line_geom(dir, i, base, stride);
      Line<T> v, o;
      load_line(tile, base, stride, v);
      line_St_t<T, 3, SP_DIR>(t, v, o);
      if (dir == D - 1) {
        const int qa = i % E, qb = i / E;
        T lt = t->lam[3][qa];
        if (D == 3) lt += t->lam[3][qb];
#pragma unroll
        for (int q = 0; q < E; ++q) o.v[q] = o.v[q] * (inv_scale * recip(t->lam[3][q] + lt));
        line_S_t<T, 3, SP_DIR>(t, o, v);
        o = v;
      }
      store_line(tile, base, stride, o);
    }
    __syncthreads();
  }
  // S along the directions before the last, ending with x as contiguous rows
#pragma unroll
  for (int dir = D - 2; dir >= 1; --dir) {
    for (int i = lane; i < nl; i += TPP) {
      int base, stride;
      line_geom(dir, i, base, stride);
      Line<T> v, o;
      load_line(tile, base, stride, v);
      line_S_t<T, 3, SP_DIR>(t, v, o);
      store_line(tile, base, stride, o);
    }
    __syncthreads();
  }
  for (int i = lane; i < nl; i += TPP) {
    const int py = i % E, pz = i / E;
    int base, stride;
    line_geom(0, i, base, stride);
    Line<T> v, o;
    load_line(tile, base, stride, v);
    line_S_t<T, 3, SP_DIR>(t, v, o);
    const long long row0 = roff + xrow_offset(2, P, py, pz);
#pragma unroll
    for (int a = 0; a < n; ++a) {
      x[row0 + a] = o.v[a];
      x[row0 + NC + a] = o.v[n + a];
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(TPP)
k_coarse(const Tab<K, T>* __restrict__ t, T inv_scale, const T* __restrict__ b, T* __restrict__ x,
         long long ndof) {
  __shared__ T tile[TS];
  coarse_body<T>(t, inv_scale, b, x, ndof, threadIdx.x, tile, blockIdx.y, true);
}

// ------------------------------------------------------- V-cycle bottom
// Levels 1 (N = 4) and 0 (N = 2) of the V-cycle in one workgroup per
// right-hand side.  A colour of level 1 has at most 2^D patches, one patch
// slot each, so colours follow each other at a barrier instead of a launch:
// pre-smoothing from x = 0 (colours ascending), residual + restriction, the
// exact coarse solve, prolongation + add, post-smoothing (descending).  Every
// patch does the arithmetic of the separate kernels.  In-place smoothers only.
constexpr int kBottomSlots = 1 << D;
constexpr int kBottomPP = kRestrictPP > smooth_pp<1>() ? kRestrictPP : smooth_pp<1>();

template <typename T>
constexpr bool bottom_fits() {
  return TPP * kBottomSlots <= 1024 && kBottomSlots * kBottomPP * (int)sizeof(T) <= 160 * 1024;
}

// the patches of one colour on the level with N cells per direction
__device__ __forceinline__ PatchGrid level_colour(int N, int colour) {
  PatchGrid g{};
  g.N = N;
  g.xcd_remap = 0;
  g.npatch = 1;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int bit = (i < D) ? (colour >> i) & 1 : 0;
    g.off[i] = bit;
    g.cnt[i] = (i < D) ? (bit ? (N - 2) / 2 : N / 2) : 1;
    g.npatch *= g.cnt[i];
  }
  return g;
}
__device__ __forceinline__ PatchGrid level1_colour(int colour) { return level_colour(4, colour); }

template <typename T>
struct BottomArgs {
  T scale1, inv_scale1, scale0_inv;
  T* x1;
  const T* b1;
  T* b0;
  T* x0;
  long long ndof1, ndof0;
};

// the stages of levels 1 and 0 (patch slot `slot`; slots past a colour's
// patches only meet the barriers)
template <typename T, int MODE>
__device__ __forceinline__ void bottom_body(const Tab<K, T>* __restrict__ t, const BottomArgs<T>& a,
                                            int slot, int lane, T* sm, int rhs) {
  constexpr int NCOL = 1 << D;
  smooth_body<T, MODE, false, true>(t, level1_colour(0), a.scale1, a.inv_scale1, a.x1, a.x1, a.b1,
                                    a.ndof1, slot, lane, sm, rhs);
  __syncthreads();
  for (int c = 1; c < NCOL; ++c) {
    smooth_body<T, MODE, false, false>(t, level1_colour(c), a.scale1, a.inv_scale1, a.x1, a.x1, a.b1,
                                       a.ndof1, slot, lane, sm, rhs);
    __syncthreads();
  }
  restrict_body<T>(t, level1_colour(0), a.scale1, a.x1, a.b1, a.b0, a.ndof1, a.ndof0, slot, lane, sm, rhs);
  __syncthreads();
  coarse_body<T>(t, a.scale0_inv, a.b0, a.x0, a.ndof0, lane, sm, rhs, slot == 0);
  __syncthreads();
  prolong_body<T>(level1_colour(0), a.x0, a.x1, a.ndof1, a.ndof0, slot, lane, sm, rhs);
  __syncthreads();
  for (int c = NCOL - 1; c >= 0; --c) {
    smooth_body<T, MODE, false, false>(t, level1_colour(c), a.scale1, a.inv_scale1, a.x1, a.x1, a.b1,
                                       a.ndof1, slot, lane, sm, rhs);
    __syncthreads();
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(TPP * kBottomSlots)
k_bottom(const Tab<K, T>* __restrict__ t, BottomArgs<T> a) {
  __shared__ T smem[kBottomSlots * kBottomPP];
  const int slot = slot_of(), lane = threadIdx.x % TPP;
  bottom_body<T, MODE>(t, a, slot, lane, smem + slot * kBottomPP, blockIdx.y);
}

// 2-D: levels 2 (N = 8) to 0 in one workgroup.  A level-2 colour has at most
// 16 patches (16 slots of E threads), so level 2's smoothing, its restriction
// and the prolongation back to it join the stages of levels 1 and 0.  Same
// bodies, so the results equal the separate kernels bit for bit.
constexpr int kBottom3Slots = 16;

template <typename T>
constexpr bool bottom3_fits() {
  return D == 2 && TPP * kBottom3Slots <= 1024 && kBottom3Slots * kBottomPP * (int)sizeof(T) <= 160 * 1024;
}

template <typename T>
struct Bottom3Args {
  BottomArgs<T> a;  // levels 1 and 0 (a.b1 is written here by the level-2 restriction)
  T scale2, inv_scale2;
  T* x2;
  const T* b2;
  T* b1w;
  long long ndof2;
};

template <typename T, int MODE>
__global__ void __launch_bounds__(TPP * kBottom3Slots)
k_bottom3(const Tab<K, T>* __restrict__ t, Bottom3Args<T> a3) {
  __shared__ T smem[kBottom3Slots * kBottomPP];
  const int slot = slot_of(), lane = threadIdx.x % TPP;
  T* sm = smem + slot * kBottomPP;
  const int rhs = blockIdx.y;
  constexpr int NCOL = 1 << D;
  smooth_body<T, MODE, false, true>(t, level_colour(8, 0), a3.scale2, a3.inv_scale2, a3.x2, a3.x2, a3.b2,
                                    a3.ndof2, slot, lane, sm, rhs);
  __syncthreads();
  for (int c = 1; c < NCOL; ++c) {
    smooth_body<T, MODE, false, false>(t, level_colour(8, c), a3.scale2, a3.inv_scale2, a3.x2, a3.x2,
                                       a3.b2, a3.ndof2, slot, lane, sm, rhs);
    __syncthreads();
  }
  restrict_body<T>(t, level_colour(8, 0), a3.scale2, a3.x2, a3.b2, a3.b1w, a3.ndof2, a3.a.ndof1, slot, lane,
                   sm, rhs);
  __syncthreads();
  bottom_body<T, MODE>(t, a3.a, slot, lane, sm, rhs);
  prolong_body<T>(level_colour(8, 0), a3.a.x1, a3.x2, a3.ndof2, a3.a.ndof1, slot, lane, sm, rhs);
  __syncthreads();
  for (int c = NCOL - 1; c >= 0; --c) {
    smooth_body<T, MODE, false, false>(t, level_colour(8, c), a3.scale2, a3.inv_scale2, a3.x2, a3.x2,
                                       a3.b2, a3.ndof2, slot, lane, sm, rhs);
    __syncthreads();
  }
}

// The same with two waves per patch in the smoothing stages (where kSplitOK
// and 2^D two-wave slots fit one workgroup: 3-D Q3): waves 2s and 2s + 1 form
// patch slot s, and the transfer and coarse stages run on the even waves while
// the odd ones meet the barriers only.  The split smoothing body gives every
// output bit for bit as the one-wave body.
constexpr bool kBottomSplitOK = kSplitOK && 2 * TPP * kBottomSlots <= 1024;

template <typename T, int MODE, bool ZERO>
__device__ __forceinline__ void bottom_smooth_half(const Tab<K, T>* __restrict__ t, int colour,
                                                   const BottomArgs<T>& a, int slot, int h, int lane,
                                                   T* sm, int rhs) {
  if (h == 0)
    smooth_split_body<T, MODE, false, ZERO, 0>(t, level1_colour(colour), a.scale1, a.inv_scale1, a.x1,
                                               a.b1, a.ndof1, slot, lane, sm, rhs);
  else
    smooth_split_body<T, MODE, false, ZERO, 1>(t, level1_colour(colour), a.scale1, a.inv_scale1, a.x1,
                                               a.b1, a.ndof1, slot, lane, sm, rhs);
}

template <typename T, int MODE>
__global__ void __launch_bounds__(2 * TPP * kBottomSlots)
k_bottom_split(const Tab<K, T>* __restrict__ t, BottomArgs<T> a) {
  static_assert(kBottomSplitOK, "two-wave slots must fit one workgroup");
  __shared__ T smem[kBottomSlots * kBottomPP];
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x / TPP);
  const int slot = w / 2, h = w % 2, lane = threadIdx.x % TPP;
  const int tslot = h == 0 ? slot : kBottomSlots;  // one-wave stages: odd waves hold no patch
  T* sm = smem + slot * kBottomPP;
  const int rhs = blockIdx.y;
  constexpr int NCOL = 1 << D;
  bottom_smooth_half<T, MODE, true>(t, 0, a, slot, h, lane, sm, rhs);
  __syncthreads();
  for (int c = 1; c < NCOL; ++c) {
    bottom_smooth_half<T, MODE, false>(t, c, a, slot, h, lane, sm, rhs);
    __syncthreads();
  }
  restrict_body<T>(t, level1_colour(0), a.scale1, a.x1, a.b1, a.b0, a.ndof1, a.ndof0, tslot, lane, sm, rhs);
  __syncthreads();
  coarse_body<T>(t, a.scale0_inv, a.b0, a.x0, a.ndof0, lane, sm, rhs, slot == 0 && h == 0);
  __syncthreads();
  prolong_body<T>(level1_colour(0), a.x0, a.x1, a.ndof1, a.ndof0, tslot, lane, sm, rhs);
  __syncthreads();
  for (int c = NCOL - 1; c >= 0; --c) {
    bottom_smooth_half<T, MODE, false>(t, c, a, slot, h, lane, sm, rhs);
    __syncthreads();
  }
}

// ------------------------------------------------------------ launchers
// Workgroup shapes the autotuner chooses between: PPB_DEFAULT patches per
// workgroup (variant 0) or twice as many (variant 1) while the workgroup stays
// within 256 threads (larger patches keep one per workgroup).
template <int V>
struct Shape {
  static constexpr int PPB =
      (V == 1 && TPP * PPB_DEFAULT * 2 > 256) ? PPB_DEFAULT : PPB_DEFAULT * (V + 1);
};

// Slots of the right-hand-side-packed shapes: at most 8 (3-D) or 16 (2-D)
// per workgroup, within 1024 threads and half the LDS of a CU.
template <typename T, int PP>
constexpr int rpack_slots() {
  int r = (D == 3) ? 8 : 16;
  while (r > 1 && (TPP * r > 1024 || r * PP * (int)sizeof(T) > 80 * 1024)) r /= 2;
  return r;
}
template <typename T>
constexpr int rpack_apply_slots() {
  return kApplyRF ? rpack_slots<T, kApplyRFPP>()
                  : rpack_slots<T, Smem<2, (D - 1) * 2 * 2 * NF>::per_patch>();
}

template <typename T, int V>
hipError_t launch_apply(const void* tab, PatchGrid g, T scale, const T* x, T* y, int nrhs,
                        long long ndof, hipStream_t s) {
  constexpr int PPB = Shape<V>::PPB;
  g.nrhs = nrhs;
  dim3 grid((g.npatch + PPB - 1) / PPB, nrhs);
  hipLaunchKernelGGL((k_apply<T, PPB>), grid, dim3(TPP * PPB), 0, s,
                     (const Tab<K, T>*)tab, g, scale, x, y, ndof);
  return hipGetLastError();
}
// shape 2: face data in registers where kApplyRF (otherwise shape 0)
template <typename T>
hipError_t launch_apply_rf(const void* tab, PatchGrid g, T scale, const T* x, T* y, int nrhs,
                           long long ndof, hipStream_t s) {
  if constexpr (!kApplyRF) {
    return launch_apply<T, 0>(tab, g, scale, x, y, nrhs, ndof, s);
  } else {
    constexpr int PPB = PPB_DEFAULT;
    g.nrhs = nrhs;
    dim3 grid((g.npatch + PPB - 1) / PPB, nrhs);
    hipLaunchKernelGGL((k_apply_rf<T, PPB>), grid, dim3(TPP * PPB), 0, s,
                       (const Tab<K, T>*)tab, g, scale, x, y, ndof);
    return hipGetLastError();
  }
}
// shape 3: one patch for several right-hand sides per workgroup (face data
// in registers in 3-D)
template <typename T>
hipError_t launch_apply_rpack(const void* tab, PatchGrid g, T scale, const T* x, T* y, int nrhs,
                              long long ndof, hipStream_t s) {
  constexpr int R = rpack_apply_slots<T>();
  g.nrhs = nrhs;
  const dim3 grid(g.npatch, (nrhs + R - 1) / R), block(TPP * R);
  if constexpr (kApplyRF)
    hipLaunchKernelGGL((k_apply_rf<T, R, true>), grid, block, 0, s, (const Tab<K, T>*)tab, g, scale, x, y,
                       ndof);
  else
    hipLaunchKernelGGL((k_apply<T, R, true>), grid, block, 0, s, (const Tab<K, T>*)tab, g, scale, x, y,
                       ndof);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_mass(const void* tab, PatchGrid g, T scale, const T* x, T* y, int nrhs,
                       long long ndof, hipStream_t s) {
  constexpr int PPB = PPB_DEFAULT;
  dim3 grid((g.npatch + PPB - 1) / PPB, nrhs);
  hipLaunchKernelGGL((k_mass<T, PPB>), grid, dim3(TPP * PPB), 0, s,
                     (const Tab<K, T>*)tab, g, scale, x, y, ndof);
  return hipGetLastError();
}
// smoother shapes: bit 0 selects the workgroup shape, bit 1 the prefetch of b,
// bit 2 two waves per patch where kSplitOK, else one patch per workgroup where
// several patches share a wave (2-D, 3-D Q1: patches of different types there
// run their fast-diagonalisation branches one after the other), else the same
// as bit 2 clear; variant 0 / 1 / 2 / 3: Dirichlet consistent / Dirichlet with
// the paper's residual / Full / clamped
constexpr bool kOnePatchShape = !kSplitOK && PPB_DEFAULT > 1;
// shapes 8..11 (bit 3): one patch for several right-hand sides per workgroup,
// bit 0 selecting the larger slot count, bit 1 the prefetch of b
template <typename T>
constexpr int rpack_smooth_slots(bool large) {
  constexpr int r = rpack_slots<T, smooth_pp<3>()>();
  return large ? r : (r > 1 ? r / 2 : 1);
}
template <typename T, int R, bool PF>
hipError_t launch_smooth_rpack(const Tab<K, T>* tb, PatchGrid g, T scale, T inv_scale, int variant,
                               int zero, const T* xin, T* xout, const T* b, int nrhs, long long ndof,
                               hipStream_t s) {
  const dim3 grid(g.npatch, (nrhs + R - 1) / R), block(TPP * R);
  if (zero) {
    if (variant == 2)
      hipLaunchKernelGGL((k_smooth<T, R, 3, false, true, true>), grid, block, 0, s, tb, g, scale,
                         inv_scale, xin, xout, b, ndof);
    else if (variant == 3)
      hipLaunchKernelGGL((k_smooth<T, R, 4, false, true, true>), grid, block, 0, s, tb, g, scale,
                         inv_scale, xout, xout, b, ndof);
    else if (variant == 1)
      hipLaunchKernelGGL((k_smooth<T, R, 2, false, true, true>), grid, block, 0, s, tb, g, scale,
                         inv_scale, xout, xout, b, ndof);
    else
      hipLaunchKernelGGL((k_smooth<T, R, 1, false, true, true>), grid, block, 0, s, tb, g, scale,
                         inv_scale, xout, xout, b, ndof);
    return hipGetLastError();
  }
  if (variant == 2)
    hipLaunchKernelGGL((k_smooth<T, R, 3, PF, false, true>), grid, block, 0, s, tb, g, scale, inv_scale,
                       xin, xout, b, ndof);
  else if (variant == 3)
    hipLaunchKernelGGL((k_smooth<T, R, 4, PF, false, true>), grid, block, 0, s, tb, g, scale, inv_scale,
                       xout, xout, b, ndof);
  else if (variant == 1)
    hipLaunchKernelGGL((k_smooth<T, R, 2, PF, false, true>), grid, block, 0, s, tb, g, scale, inv_scale,
                       xout, xout, b, ndof);
  else
    hipLaunchKernelGGL((k_smooth<T, R, 1, PF, false, true>), grid, block, 0, s, tb, g, scale, inv_scale,
                       xout, xout, b, ndof);
  return hipGetLastError();
}
template <typename T, int V>
hipError_t launch_smooth(const void* tab, PatchGrid g, T scale, T inv_scale, int variant, int zero,
                         const T* xin, T* xout, const T* b, int nrhs, long long ndof, hipStream_t s) {
  constexpr int PPB = (kOnePatchShape && (V & 4)) ? 1 : Shape<(V & 1)>::PPB;
  constexpr bool PF = (V & 2) != 0;
  constexpr bool SPLIT = (V & 4) != 0 && kSplitOK;
  g.nrhs = nrhs;
  const Tab<K, T>* tb = (const Tab<K, T>*)tab;
  if constexpr ((V & 8) != 0) {
    constexpr int R = rpack_smooth_slots<T>((V & 1) != 0);
    return launch_smooth_rpack<T, R, PF>(tb, g, scale, inv_scale, variant, zero, xin, xout, b, nrhs, ndof,
                                         s);
  }
  dim3 grid((g.npatch + PPB - 1) / PPB, nrhs);
  if constexpr (SPLIT) {
    if (variant != 2) {
      const dim3 block(2 * TPP * PPB);
      if (zero) {
        if (variant == 3)
          hipLaunchKernelGGL((k_smooth_split<T, PPB, 4, false, true>), grid, block, 0, s, tb, g, scale,
                             inv_scale, xout, b, ndof);
        else if (variant == 1)
          hipLaunchKernelGGL((k_smooth_split<T, PPB, 2, false, true>), grid, block, 0, s, tb, g, scale,
                             inv_scale, xout, b, ndof);
        else
          hipLaunchKernelGGL((k_smooth_split<T, PPB, 1, false, true>), grid, block, 0, s, tb, g, scale,
                             inv_scale, xout, b, ndof);
      } else if (variant == 3) {
        hipLaunchKernelGGL((k_smooth_split<T, PPB, 4, PF>), grid, block, 0, s, tb, g, scale, inv_scale,
                           xout, b, ndof);
      } else if (variant == 1) {
        hipLaunchKernelGGL((k_smooth_split<T, PPB, 2, PF>), grid, block, 0, s, tb, g, scale, inv_scale,
                           xout, b, ndof);
      } else {
        hipLaunchKernelGGL((k_smooth_split<T, PPB, 1, PF>), grid, block, 0, s, tb, g, scale, inv_scale,
                           xout, b, ndof);
      }
      return hipGetLastError();
    }
  }
  if (zero) {  // x = 0, colour 0: the residual is b, no prefetch needed
    if (variant == 2)
      hipLaunchKernelGGL((k_smooth<T, PPB, 3, false, true>), grid, dim3(TPP * PPB), 0, s, tb, g,
                         scale, inv_scale, xin, xout, b, ndof);
    else if (variant == 3)
      hipLaunchKernelGGL((k_smooth<T, PPB, 4, false, true>), grid, dim3(TPP * PPB), 0, s, tb, g,
                         scale, inv_scale, xout, xout, b, ndof);
    else if (variant == 1)
      hipLaunchKernelGGL((k_smooth<T, PPB, 2, false, true>), grid, dim3(TPP * PPB), 0, s, tb, g,
                         scale, inv_scale, xout, xout, b, ndof);
    else
      hipLaunchKernelGGL((k_smooth<T, PPB, 1, false, true>), grid, dim3(TPP * PPB), 0, s, tb, g,
                         scale, inv_scale, xout, xout, b, ndof);
    return hipGetLastError();
  }
  if (variant == 2)
    hipLaunchKernelGGL((k_smooth<T, PPB, 3, PF>), grid, dim3(TPP * PPB), 0, s, tb, g, scale,
                       inv_scale, xin, xout, b, ndof);
  else if (variant == 3)
    hipLaunchKernelGGL((k_smooth<T, PPB, 4, PF>), grid, dim3(TPP * PPB), 0, s, tb, g, scale,
                       inv_scale, xout, xout, b, ndof);
  else if (variant == 1)
    hipLaunchKernelGGL((k_smooth<T, PPB, 2, PF>), grid, dim3(TPP * PPB), 0, s, tb, g, scale,
                       inv_scale, xout, xout, b, ndof);
  else
    hipLaunchKernelGGL((k_smooth<T, PPB, 1, PF>), grid, dim3(TPP * PPB), 0, s, tb, g, scale,
                       inv_scale, xout, xout, b, ndof);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_restrict(const void* tab, PatchGrid g, T scale, const T* x, const T* b, T* bc,
                           int nrhs, long long ndof, long long ndof_c, hipStream_t s) {
  constexpr int PPB = PPB_DEFAULT;
  dim3 grid((g.npatch + PPB - 1) / PPB, nrhs);
  if constexpr (kRestrictOnApplyRF)
    hipLaunchKernelGGL((k_restrict_rf<T, PPB>), grid, dim3(TPP * PPB), 0, s,
                       (const Tab<K, T>*)tab, g, scale, x, b, bc, ndof, ndof_c);
  else
    hipLaunchKernelGGL((k_restrict<T, PPB>), grid, dim3(TPP * PPB), 0, s,
                       (const Tab<K, T>*)tab, g, scale, x, b, bc, ndof, ndof_c);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_prolong(const void* tab, PatchGrid g, const T* xc, T* x, int nrhs,
                          long long ndof, long long ndof_c, hipStream_t s) {
  constexpr int PPB = PPB_DEFAULT;
  dim3 grid((g.npatch + PPB - 1) / PPB, nrhs);
  hipLaunchKernelGGL((k_prolong<T, PPB>), grid, dim3(TPP * PPB), 0, s,
                     (const Tab<K, T>*)tab, g, xc, x, ndof, ndof_c);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_coarse(const void* tab, T inv_scale, const T* b, T* x, int nrhs, long long ndof,
                         hipStream_t s) {
  dim3 grid(1, nrhs);
  hipLaunchKernelGGL((k_coarse<T>), grid, dim3(TPP), 0, s, (const Tab<K, T>*)tab, inv_scale, b, x,
                     ndof);
  return hipGetLastError();
}

// variant 0 / 1 / 3 (in-place smoothers); the Full kernel is not fused.
// split: two waves per patch in the smoothing stages where kBottomSplitOK.
template <typename T>
hipError_t launch_bottom(const void* tab, int variant, int split, T scale1, T inv_scale1, T inv_scale0,
                         T* x1, const T* b1, T* b0, T* x0, int nrhs, long long ndof1, long long ndof0,
                         hipStream_t s) {
  if constexpr (!bottom_fits<T>()) {
    return hipErrorInvalidConfiguration;
  } else {
    const BottomArgs<T> a{scale1, inv_scale1, inv_scale0, x1, b1, b0, x0, ndof1, ndof0};
    const Tab<K, T>* tb = (const Tab<K, T>*)tab;
    const dim3 grid(1, nrhs), block(TPP * kBottomSlots);
    if constexpr (kBottomSplitOK) {
      if (split) {
        const dim3 block2(2 * TPP * kBottomSlots);
        if (variant == 0) hipLaunchKernelGGL((k_bottom_split<T, 1>), grid, block2, 0, s, tb, a);
        else if (variant == 1) hipLaunchKernelGGL((k_bottom_split<T, 2>), grid, block2, 0, s, tb, a);
        else if (variant == 3) hipLaunchKernelGGL((k_bottom_split<T, 4>), grid, block2, 0, s, tb, a);
        else return hipErrorInvalidValue;
        return hipGetLastError();
      }
    }
    if (variant == 0) hipLaunchKernelGGL((k_bottom<T, 1>), grid, block, 0, s, tb, a);
    else if (variant == 1) hipLaunchKernelGGL((k_bottom<T, 2>), grid, block, 0, s, tb, a);
    else if (variant == 3) hipLaunchKernelGGL((k_bottom<T, 4>), grid, block, 0, s, tb, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
}

// levels 2, 1, 0 in one launch (2-D; variants 0 / 1 / 3)
template <typename T>
hipError_t launch_bottom3(const void* tab, int variant, T scale2, T inv_scale2, T scale1, T inv_scale1,
                          T inv_scale0, T* x2, const T* b2, T* x1, T* b1, T* b0, T* x0, int nrhs,
                          long long ndof2, long long ndof1, long long ndof0, hipStream_t s) {
  if constexpr (!bottom3_fits<T>()) {
    return hipErrorInvalidConfiguration;
  } else {
    Bottom3Args<T> a3;
    a3.a = BottomArgs<T>{scale1, inv_scale1, inv_scale0, x1, b1, b0, x0, ndof1, ndof0};
    a3.scale2 = scale2;
    a3.inv_scale2 = inv_scale2;
    a3.x2 = x2;
    a3.b2 = b2;
    a3.b1w = b1;
    a3.ndof2 = ndof2;
    const Tab<K, T>* tb = (const Tab<K, T>*)tab;
    const dim3 grid(1, nrhs), block(TPP * kBottom3Slots);
    if (variant == 0) hipLaunchKernelGGL((k_bottom3<T, 1>), grid, block, 0, s, tb, a3);
    else if (variant == 1) hipLaunchKernelGGL((k_bottom3<T, 2>), grid, block, 0, s, tb, a3);
    else if (variant == 3) hipLaunchKernelGGL((k_bottom3<T, 4>), grid, block, 0, s, tb, a3);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
}

template <typename T>
KernelSet<T> make_set() {
  KernelSet<T> k;
  k.apply[0] = &launch_apply<T, 0>;
  k.apply[1] = &launch_apply<T, 1>;
  k.apply[2] = &launch_apply_rf<T>;
  k.apply[3] = &launch_apply_rpack<T>;
  k.apply_rf = kApplyRF ? 1 : 0;
  k.apply_rpack = rpack_apply_slots<T>() > 1 ? 1 : 0;
  k.smooth_rpack = rpack_smooth_slots<T>(true) > 1 ? 1 : 0;
  k.mass = &launch_mass<T>;
  k.smooth[0] = &launch_smooth<T, 0>;
  k.smooth[1] = &launch_smooth<T, 1>;
  k.smooth[2] = &launch_smooth<T, 2>;
  k.smooth[3] = &launch_smooth<T, 3>;
  k.smooth[4] = &launch_smooth<T, 4>;
  k.smooth[5] = &launch_smooth<T, 5>;
  k.smooth[6] = &launch_smooth<T, 6>;
  k.smooth[7] = &launch_smooth<T, 7>;
  k.smooth[8] = &launch_smooth<T, 8>;
  k.smooth[9] = &launch_smooth<T, 9>;
  k.smooth[10] = &launch_smooth<T, 10>;
  k.smooth[11] = &launch_smooth<T, 11>;
  k.smooth_split = (kSplitOK || kOnePatchShape) ? 1 : 0;
  k.smooth_hi_full = kOnePatchShape ? 1 : 0;
  k.restrict_residual = &launch_restrict<T>;
  k.prolongate_add = &launch_prolong<T>;
  k.coarse = &launch_coarse<T>;
  k.bottom = bottom_fits<T>() ? &launch_bottom<T> : nullptr;
  k.bottom_split = (bottom_fits<T>() && kBottomSplitOK) ? 1 : 0;
  k.bottom3 = bottom3_fits<T>() ? &launch_bottom3<T> : nullptr;
  return k;
}

}  // namespace
}  // namespace dgmg

#define DGMG_CAT2(a, b, c, d) a##b##c##d
#define DGMG_ENTRY(Dv, Kv) DGMG_CAT2(dgmg_kernels_d, Dv, _k, Kv)
extern "C" void DGMG_ENTRY(DGMG_D, DGMG_K)(dgmg::KernelEntry* e) {
  e->dim = DGMG_D;
  e->degree = DGMG_K;
  e->f64 = dgmg::make_set<double>();
  e->f32 = dgmg::make_set<float>();
}
