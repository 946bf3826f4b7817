// Patch-tile kernels of the SIPG multigrid hot path for one (dimension D,
// degree K) pair, selected by -DDGMG_D=<2|3> -DDGMG_K=<1..7>; the build
// compiles this file once per pair.
//
// Every kernel works on "patches": the 2^D cells with coordinates lo_i and
// lo_i + 1 in each direction i.  A patch carries E = 2(K+1) nodes per
// direction (patch-local index p = n c + a for cell c in {0,1}, node a).  One
// workgroup owns PPB patches; each patch's node tile sits in LDS with padded
// strides (SY, SZ).  Work inside a patch proceeds in phases separated by
// barriers; in a phase along direction `dir` each thread owns one 1-D line of
// the tile (all other coordinates fixed), pulls it into registers, contracts
// it with the 1-D matrices (wave-uniform, read through scalar loads from the
// Tab struct) and writes the result back to its own line.
//
// Operator (Sec. 2.2): on a Cartesian mesh A = sum_i (x)(M .. L_i .. M), with
// reference matrices (h = 1) and A_h = kappa h^(D-2) A_ref.  The 1-D SIPG
// operator restricted to the patch is applied per cell block (Lc) plus rank-2
// face couplings: for a cell with trace t and derivative g of its neighbour
// across a face, the rows pick up e (alpha) + d (beta) with
//   left neighbour  (its x=1 side):  alpha = g/2 - sigma t, beta = -t/2 (e0, d0)
//   right neighbour (its x=0 side):  alpha = -sigma t - g/2, beta =  t/2 (e1, d1)
// and on a domain-boundary face the Nitsche correction of the cell block,
//   x=0: alpha = (d0.v)/2, beta = v_0/2;   x=1: alpha = -(d1.v)/2, beta = -v_k/2.
// Face data of the outside neighbours ("ext") is gathered per face node in
// the load phase; faces normal to y and z are pre-contracted with the
// tangential masses so that the sum-factorised order
//   a = M_x x, b = L_x x;  c = M_y b + L_y a, d = M_y a;  y = M_z c + L_z d
// needs only one pass per direction.
#include "dgmg_internal.h"

#ifndef DGMG_D
#error "DGMG_D must be defined"
#endif
#ifndef DGMG_K
#error "DGMG_K must be defined"
#endif

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
constexpr int SZ = (D == 3) ? E * SY + 1 : 0;
constexpr int TS = (D == 2) ? E * SY : E * SZ;      // padded tile size
constexpr int NEXT = D * 2 * 2 * NL;                // ext face data per patch

// threads per patch (one per line) and patches per workgroup
constexpr int TPP = NL;
constexpr int PPB_DEFAULT = (D == 3)
    ? (K == 1 ? 4 : K == 2 ? 7 : K == 3 ? 2 : K == 4 ? 2 : 1)
    : (K == 1 ? 16 : K == 2 ? 10 : K == 3 ? 8 : K == 4 ? 6 : K == 5 ? 5 : 4);

__host__ __device__ constexpr int cpow(int b, int e) { return e == 0 ? 1 : b * cpow(b, e - 1); }

__device__ __forceinline__ int toff(int px, int py, int pz) { return px + py * SY + pz * SZ; }

// base offset and stride of line l along direction dir
__device__ __forceinline__ void line_geom(int dir, int l, int& base, int& stride) {
  const int a = l % E, b = l / E;
  if (dir == 0) { base = a * SY + b * SZ; stride = 1; }
  else if (dir == 1) { base = a + b * SZ; stride = SY; }
  else { base = a + b * SY; stride = SZ; }
}

__device__ __forceinline__ int ext_idx(int dir, int side, int comp, int l) {
  return ((dir * 2 + side) * 2 + comp) * NL + l;
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

// o = blockdiag(M, M) v
template <typename T>
__device__ __forceinline__ void line_mass(const Tab<K, T>* __restrict__ t, const Line<T>& v, Line<T>& o) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int mu = 0; mu < n; ++mu) {
      T s = T(0);
#pragma unroll
      for (int nu = 0; nu < n; ++nu) s += t->M[mu * n + nu] * v.v[c * n + nu];
      o.v[c * n + mu] = s;
    }
}

// o (+)= 1-D SIPG on the patch line v with outside couplings (aL, bL, aR, bR)
template <typename T, bool ACC>
__device__ __forceinline__ void line_sipg(const Tab<K, T>* __restrict__ t, const Line<T>& v,
                                          T aL, T bL, T aR, T bR, Line<T>& o) {
  const T sg = t->sigma;
  const T half = T(0.5);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int mu = 0; mu < n; ++mu) {
      T s = ACC ? o.v[c * n + mu] : T(0);
#pragma unroll
      for (int nu = 0; nu < n; ++nu) s += t->Lc[mu * n + nu] * v.v[c * n + nu];
      o.v[c * n + mu] = s;
    }
  // coupling across the face between the two patch cells
  const T tR = v.v[n];      // trace of the right cell at its x=0 side
  const T tL = v.v[n - 1];  // trace of the left cell at its x=1 side
  T gR = T(0), gL = T(0);
#pragma unroll
  for (int j = 0; j < n; ++j) {
    gR += t->d0[j] * v.v[n + j];
    gL += t->d1[j] * v.v[j];
  }
  const T bLc = half * tR;   // beta seen by the left cell from its right neighbour
  const T bRc = -half * tL;  // beta seen by the right cell from its left neighbour
  o.v[0] += aL;
  o.v[n - 1] += -sg * tR - half * gR;
  o.v[n] += half * gL - sg * tL;
  o.v[E - 1] += aR;
#pragma unroll
  for (int mu = 0; mu < n; ++mu) {
    o.v[mu] += t->d0[mu] * bL + t->d1[mu] * bLc;
    o.v[n + mu] += t->d0[mu] * bRc + t->d1[mu] * bR;
  }
}

// Fast-diagonalisation contractions for patch type TY (padded S: rows p in
// [PLO, PHI) and columns q < QN are the only non-zeros).
template <int TY> struct FDB;
template <> struct FDB<0> { static constexpr int PLO = 1, PHI = E - 1, QN = E - 2; };
template <> struct FDB<1> { static constexpr int PLO = 0, PHI = E - 1, QN = E - 1; };
template <> struct FDB<2> { static constexpr int PLO = 1, PHI = E, QN = E - 1; };
template <> struct FDB<3> { static constexpr int PLO = 0, PHI = E, QN = E; };

// o[q] = sum_p S[p][q] v[p]
template <typename T, int TY>
__device__ __forceinline__ void line_St_t(const Tab<K, T>* __restrict__ t, const Line<T>& v, Line<T>& o) {
  using B = FDB<TY>;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    T s = T(0);
    if (q < B::QN) {
#pragma unroll
      for (int p = B::PLO; p < B::PHI; ++p) s += t->S[TY][p * E + q] * v.v[p];
    }
    o.v[q] = s;
  }
}
// o[p] = sum_q S[p][q] v[q]
template <typename T, int TY>
__device__ __forceinline__ void line_S_t(const Tab<K, T>* __restrict__ t, const Line<T>& v, Line<T>& o) {
  using B = FDB<TY>;
#pragma unroll
  for (int p = 0; p < E; ++p) {
    T s = T(0);
    if (p >= B::PLO && p < B::PHI) {
#pragma unroll
      for (int q = 0; q < B::QN; ++q) s += t->S[TY][p * E + q] * v.v[q];
    }
    o.v[p] = s;
  }
}
template <typename T>
__device__ __forceinline__ void line_St(const Tab<K, T>* __restrict__ t, int ty, const Line<T>& v, Line<T>& o) {
  switch (ty) {
    case 0: line_St_t<T, 0>(t, v, o); break;
    case 1: line_St_t<T, 1>(t, v, o); break;
    case 2: line_St_t<T, 2>(t, v, o); break;
    default: line_St_t<T, 3>(t, v, o); break;
  }
}
template <typename T>
__device__ __forceinline__ void line_S(const Tab<K, T>* __restrict__ t, int ty, const Line<T>& v, Line<T>& o) {
  switch (ty) {
    case 0: line_S_t<T, 0>(t, v, o); break;
    case 1: line_S_t<T, 1>(t, v, o); break;
    case 2: line_S_t<T, 2>(t, v, o); break;
    default: line_S_t<T, 3>(t, v, o); break;
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

// Copy the patch's 2^D cells from global to the LDS tile (coalesced per cell).
template <typename T>
__device__ __forceinline__ void load_tile(const T* __restrict__ x, int N, const PatchPos& P,
                                          int lane, T* tile) {
  for (int i = lane; i < NCP * NC; i += TPP) {
    const int c = i / NC, loc = i % NC;
    const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
    const int ax = loc % n, ay = (loc / n) % n, az = loc / (n * n);
    const long long cell = cell_index(N, P.lo[0] + cx, P.lo[1] + cy, (D == 3) ? P.lo[2] + cz : 0);
    tile[toff(cx * n + ax, cy * n + ay, cz * n + az)] = x[cell * NC + loc];
  }
}

// Face data of the 2D sides of the patch.  For face node l of direction dir,
// side s: the neighbour cell across the patch boundary (or, on the domain
// boundary, the patch's own cell for the Nitsche correction) is read along
// dir.  MODE 0: alpha and beta (operator rows on all patch nodes);
// MODE 1: smoother, beta only for interior faces (alpha acts on dropped rows);
// MODE 2: paper-literal smoother, interior faces ignored.
template <typename T, int MODE>
__device__ __forceinline__ void load_ext(const Tab<K, T>* __restrict__ t, const T* __restrict__ x,
                                         int N, const PatchPos& P, int lane, T* ext) {
  const T half = T(0.5);
  const T sg = t->sigma;
  for (int i = lane; i < D * 2 * NL; i += TPP) {
    const int l = i % NL;
    const int side = (i / NL) & 1;
    const int dir = i / (2 * NL);
    // tangential tile coordinates of face node l
    int pc[3] = {0, 0, 0};
    {
      const int a = l % E, b = l / E;
      if (dir == 0) { pc[1] = a; pc[2] = b; }
      else if (dir == 1) { pc[0] = a; pc[2] = b; }
      else { pc[0] = a; pc[1] = b; }
    }
    int cc[3], ac[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) { cc[j] = P.lo[j] + pc[j] / n; ac[j] = pc[j] % n; }
    const int nb = (side == 0) ? P.lo[dir] - 1 : P.lo[dir] + 2;
    const bool interior = (nb >= 0 && nb < N);
    const int strideN = (dir == 0) ? 1 : (dir == 1) ? n : n * n;
    T alpha = T(0), beta = T(0);
    if (interior) {
      if (MODE != 2) {
        cc[dir] = nb;
        ac[dir] = 0;
        const long long base = cell_index(N, cc[0], cc[1], cc[2]) * NC + ac[0] + n * (ac[1] + n * ac[2]);
        const T tr = x[base + (long long)((side == 0) ? K : 0) * strideN];
        if (MODE == 0) {
          T g = T(0);
#pragma unroll
          for (int j = 0; j < n; ++j) g += ((side == 0) ? t->d1[j] : t->d0[j]) * x[base + (long long)j * strideN];
          alpha = (side == 0) ? (half * g - sg * tr) : (-sg * tr - half * g);
        }
        beta = (side == 0) ? -half * tr : half * tr;
      }
    } else {
      cc[dir] = (side == 0) ? P.lo[dir] : P.lo[dir] + 1;
      ac[dir] = 0;
      const long long base = cell_index(N, cc[0], cc[1], cc[2]) * NC + ac[0] + n * (ac[1] + n * ac[2]);
      T g = T(0);
#pragma unroll
      for (int j = 0; j < n; ++j) g += ((side == 0) ? t->d0[j] : t->d1[j]) * x[base + (long long)j * strideN];
      const T tr = x[base + (long long)((side == 0) ? 0 : K) * strideN];
      alpha = (side == 0) ? half * g : -half * g;
      beta = (side == 0) ? half * tr : -half * tr;
    }
    ext[ext_idx(dir, side, 0, l)] = alpha;
    ext[ext_idx(dir, side, 1, l)] = beta;
  }
}

// Tangential mass contraction of the ext arrays, lines along direction
// `along` of faces normal to `dir` (face index l = a + E b).
template <typename T>
__device__ __forceinline__ void ext_mass_line(const Tab<K, T>* __restrict__ t, T* ext, int dir,
                                              int along_first, int j) {
  // j enumerates (side, comp, fixed coordinate): 4 * E lines
  const int fixed = j % E;
  const int sc = j / E;  // side*2 + comp
  T* a = ext + (dir * 4 + sc) * NL;
  const int base = along_first ? fixed * E : fixed;
  const int stride = along_first ? 1 : E;
  Line<T> v, o;
#pragma unroll
  for (int p = 0; p < E; ++p) v.v[p] = a[base + p * stride];
  line_mass<T>(t, v, o);
#pragma unroll
  for (int p = 0; p < E; ++p) a[base + p * stride] = o.v[p];
}

// The three (two) sum-factorisation passes of y = A_ref x on the patch tile.
// After the call the tile A holds, for D = 3, nothing useful, and the output
// lines are handed to `emit(line index, Line)` in the last (z / y) phase.
// bufA holds x on entry; bufB is scratch.
template <typename T, typename Emit>
__device__ __forceinline__ void operator_passes(const Tab<K, T>* __restrict__ t, T* bufA, T* bufB,
                                                T* ext, int lane, bool active, Emit emit) {
  // `active` gates the work only: every thread of the block meets every barrier.
  // X phase: a = M_x x -> A, b = L_x x -> B; ext of y/z faces: M_x
  {
    const int nextl = (D == 3) ? 8 * E : 4;
    for (int i = lane; active && i < NL + nextl; i += TPP) {
      if (i < NL) {
        int base, stride;
        line_geom(0, i, base, stride);
        Line<T> v, a, b;
        load_line(bufA, base, stride, v);
        line_mass<T>(t, v, a);
        line_sipg<T, false>(t, v, ext[ext_idx(0, 0, 0, i)], ext[ext_idx(0, 0, 1, i)],
                            ext[ext_idx(0, 1, 0, i)], ext[ext_idx(0, 1, 1, i)], b);
        store_line(bufA, base, stride, a);
        store_line(bufB, base, stride, b);
      } else {
        const int j = i - NL;
        if (D == 3) {
          if (j < 4 * E) ext_mass_line<T>(t, ext, 1, 1, j);
          else ext_mass_line<T>(t, ext, 2, 1, j - 4 * E);
        } else {
          // 2-D: faces normal to y are indexed by px only; 4 lines of length E
          T* a = ext + (1 * 4 + j) * NL;
          Line<T> v, o;
#pragma unroll
          for (int p = 0; p < E; ++p) v.v[p] = a[p];
          line_mass<T>(t, v, o);
#pragma unroll
          for (int p = 0; p < E; ++p) a[p] = o.v[p];
        }
      }
    }
  }
  __syncthreads();
  if constexpr (D == 3) {
    // Y phase: c = M_y b + L_y a -> B, d = M_y a -> A; ext of z faces: M_y
    for (int i = lane; active && i < NL + 4 * E; i += TPP) {
      if (i < NL) {
        int base, stride;
        line_geom(1, i, base, stride);
        Line<T> a, b, c, d;
        load_line(bufA, base, stride, a);
        load_line(bufB, base, stride, b);
        line_mass<T>(t, b, c);
        line_sipg<T, true>(t, a, ext[ext_idx(1, 0, 0, i)], ext[ext_idx(1, 0, 1, i)],
                           ext[ext_idx(1, 1, 0, i)], ext[ext_idx(1, 1, 1, i)], c);
        line_mass<T>(t, a, d);
        store_line(bufB, base, stride, c);
        store_line(bufA, base, stride, d);
      } else {
        ext_mass_line<T>(t, ext, 2, 0, i - NL);
      }
    }
    __syncthreads();
    // Z phase: y = M_z c + L_z d
    for (int i = lane; active && i < NL; i += TPP) {
      int base, stride;
      line_geom(2, i, base, stride);
      Line<T> c, d, y;
      load_line(bufB, base, stride, c);
      load_line(bufA, base, stride, d);
      line_mass<T>(t, c, y);
      line_sipg<T, true>(t, d, ext[ext_idx(2, 0, 0, i)], ext[ext_idx(2, 0, 1, i)],
                         ext[ext_idx(2, 1, 0, i)], ext[ext_idx(2, 1, 1, i)], y);
      emit(i, base, stride, y);
    }
  } else {
    // Y phase (2-D): y = M_y b + L_y a
    for (int i = lane; active && i < NL; i += TPP) {
      int base, stride;
      line_geom(1, i, base, stride);
      Line<T> a, b, y;
      load_line(bufA, base, stride, a);
      load_line(bufB, base, stride, b);
      line_mass<T>(t, b, y);
      line_sipg<T, true>(t, a, ext[ext_idx(1, 0, 0, i)], ext[ext_idx(1, 0, 1, i)],
                         ext[ext_idx(1, 1, 0, i)], ext[ext_idx(1, 1, 1, i)], y);
      emit(i, base, stride, y);
    }
  }
}

// Coalesced write of the tile back to the patch's cells (y = tile, or
// y += tile when ADD).
template <typename T, bool ADD>
__device__ __forceinline__ void store_tile(T* __restrict__ y, int N, const PatchPos& P, int lane,
                                           const T* tile) {
  for (int i = lane; i < NCP * NC; i += TPP) {
    const int c = i / NC, loc = i % NC;
    const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
    const int ax = loc % n, ay = (loc / n) % n, az = loc / (n * n);
    const long long cell = cell_index(N, P.lo[0] + cx, P.lo[1] + cy, (D == 3) ? P.lo[2] + cz : 0);
    const T v = tile[toff(cx * n + ax, cy * n + ay, cz * n + az)];
    if (ADD) y[cell * NC + loc] += v;
    else y[cell * NC + loc] = v;
  }
}

template <int NB, bool EXT, typename T>
struct Smem {
  static constexpr int per_patch = NB * TS + (EXT ? NEXT : 0);
};

// ---------------------------------------------------------------- apply
template <typename T, int PPB>
__global__ void __launch_bounds__(TPP * PPB)
k_apply(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, const T* __restrict__ x,
        T* __restrict__ y, long long ndof) {
  constexpr int PP = Smem<2, true, T>::per_patch;
  __shared__ T smem[PPB * PP];
  const int slot = threadIdx.x / TPP, lane = threadIdx.x % TPP;
  const int pid = blockIdx.x * PPB + slot;
  const bool active = pid < g.npatch;
  T* bufA = smem + slot * PP;
  T* bufB = bufA + TS;
  T* ext = bufB + TS;
  const long long roff = (long long)blockIdx.y * ndof;
  const T* xr = x + roff;
  T* yr = y + roff;
  PatchPos P = patch_pos(g, active ? pid : 0);
  if (active) {
    load_tile<T>(xr, g.N, P, lane, bufA);
    load_ext<T, 0>(t, xr, g.N, P, lane, ext);
  }
  __syncthreads();
  operator_passes<T>(t, bufA, bufB, ext, lane, active, [&](int, int base, int stride, const Line<T>& v) {
#pragma unroll
    for (int p = 0; p < E; ++p) bufA[base + p * stride] = scale * v.v[p];
  });
  __syncthreads();
  if (active) store_tile<T, false>(yr, g.N, P, lane, bufA);
}

// ----------------------------------------------------------------- mass
template <typename T, int PPB>
__global__ void __launch_bounds__(TPP * PPB)
k_mass(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, const T* __restrict__ x,
       T* __restrict__ y, long long ndof) {
  __shared__ T smem[PPB * TS];
  const int slot = threadIdx.x / TPP, lane = threadIdx.x % TPP;
  const int pid = blockIdx.x * PPB + slot;
  const bool active = pid < g.npatch;
  T* tile = smem + slot * TS;
  const long long roff = (long long)blockIdx.y * ndof;
  PatchPos P = patch_pos(g, active ? pid : 0);
  if (active) load_tile<T>(x + roff, g.N, P, lane, tile);
  __syncthreads();
#pragma unroll
  for (int dir = 0; dir < D; ++dir) {
    if (active) {
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(dir, i, base, stride);
        Line<T> v, o;
        load_line(tile, base, stride, v);
        line_mass<T>(t, v, o);
        if (dir == D - 1) {
#pragma unroll
          for (int p = 0; p < E; ++p) o.v[p] *= scale;
        }
        store_line(tile, base, stride, o);
      }
    }
    __syncthreads();
  }
  if (active) store_tile<T, false>(y + roff, g.N, P, lane, tile);
}

// -------------------------------------------------------------- smoother
// One colour of Alg. 1: local residual on the patch, then fast
// diagonalisation x|V_j += (x)S (sum lambda)^{-1} (x)S^T r_j.
template <typename T, int PPB, int MODE>
__global__ void __launch_bounds__(TPP * PPB)
k_smooth(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, T inv_scale, T* __restrict__ x,
         const T* __restrict__ b, long long ndof) {
  constexpr int PP = Smem<3, true, T>::per_patch;
  __shared__ T smem[PPB * PP];
  const int slot = threadIdx.x / TPP, lane = threadIdx.x % TPP;
  const int pid = blockIdx.x * PPB + slot;
  const bool active = pid < g.npatch;
  T* bufA = smem + slot * PP;
  T* bufB = bufA + TS;
  T* bufC = bufB + TS;
  T* ext = bufC + TS;
  const long long roff = (long long)blockIdx.y * ndof;
  T* xr = x + roff;
  const T* br = b + roff;
  PatchPos P = patch_pos(g, active ? pid : 0);
  if (active) {
    load_tile<T>(xr, g.N, P, lane, bufA);
    load_tile<T>(br, g.N, P, lane, bufC);
    load_ext<T, MODE>(t, xr, g.N, P, lane, ext);
  }
  __syncthreads();
  const int tyx = P.ty[0], tyy = P.ty[1], tyz = P.ty[2];
  // residual lines of the last operator pass, contracted with S^T of that
  // direction and parked in A
  auto emit = [&](int, int base, int stride, const Line<T>& v) {
    Line<T> r, o;
#pragma unroll
    for (int p = 0; p < E; ++p) r.v[p] = bufC[base + p * stride] - scale * v.v[p];
    line_St<T>(t, (D == 3) ? tyz : tyy, r, o);
    store_line(bufA, base, stride, o);
  };
  operator_passes<T>(t, bufA, bufB, ext, lane, active, emit);
  __syncthreads();
  if constexpr (D == 3) {
    // S_y^T
    if (active)
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(1, i, base, stride);
        Line<T> v, o;
        load_line(bufA, base, stride, v);
        line_St<T>(t, tyy, v, o);
        store_line(bufA, base, stride, o);
      }
    __syncthreads();
  }
  // S_x^T, scale by 1/(sum lambda), S_x
  if (active)
    for (int i = lane; i < NL; i += TPP) {
      int base, stride;
      line_geom(0, i, base, stride);
      const int qy = i % E, qz = i / E;
      T lt = t->lam[tyy][qy];
      if (D == 3) lt += t->lam[tyz][qz];
      Line<T> v, o;
      load_line(bufA, base, stride, v);
      line_St<T>(t, tyx, v, o);
#pragma unroll
      for (int q = 0; q < E; ++q) o.v[q] = o.v[q] * (inv_scale / (t->lam[tyx][q] + lt));
      line_S<T>(t, tyx, o, v);
      store_line(bufA, base, stride, v);
    }
  __syncthreads();
  // S_y (and S_z)
#pragma unroll
  for (int dir = 1; dir < D; ++dir) {
    if (active)
      for (int i = lane; i < NL; i += TPP) {
        int base, stride;
        line_geom(dir, i, base, stride);
        Line<T> v, o;
        load_line(bufA, base, stride, v);
        line_S<T>(t, dir == 1 ? tyy : tyz, v, o);
        store_line(bufA, base, stride, o);
      }
    __syncthreads();
  }
  // x += delta on V_j (dropped nodes have zero rows in S, so delta = 0 there;
  // they are skipped to leave other patches' reads untouched)
  if (active) {
    for (int i = lane; i < NCP * NC; i += TPP) {
      const int c = i / NC, loc = i % NC;
      const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
      const int px = cx * n + loc % n, py = cy * n + (loc / n) % n, pz = cz * n + loc / (n * n);
      const bool keep = (px > 0 || (tyx & 1)) && (px < E - 1 || (tyx & 2)) &&
                        (py > 0 || (tyy & 1)) && (py < E - 1 || (tyy & 2)) &&
                        (D == 2 || ((pz > 0 || (tyz & 1)) && (pz < E - 1 || (tyz & 2))));
      if (keep) {
        const long long cell = cell_index(g.N, P.lo[0] + cx, P.lo[1] + cy, (D == 3) ? P.lo[2] + cz : 0);
        xr[cell * NC + loc] += bufA[toff(px, py, pz)];
      }
    }
  }
}

// ------------------------------------------------- residual + restriction
// bc = P^T (b - A x): the colour-0 patch of level l is the set of children of
// one coarse cell, so its tile residual contracts with the stacked P^T per
// direction straight into that coarse cell.
template <typename T, int PPB>
__global__ void __launch_bounds__(TPP * PPB)
k_restrict(const Tab<K, T>* __restrict__ t, PatchGrid g, T scale, const T* __restrict__ x,
           const T* __restrict__ b, T* __restrict__ bc, long long ndof, long long ndof_c) {
  constexpr int PP = Smem<3, true, T>::per_patch;
  __shared__ T smem[PPB * PP];
  const int slot = threadIdx.x / TPP, lane = threadIdx.x % TPP;
  const int pid = blockIdx.x * PPB + slot;
  const bool active = pid < g.npatch;
  T* bufA = smem + slot * PP;
  T* bufB = bufA + TS;
  T* bufC = bufB + TS;
  T* ext = bufC + TS;
  const long long roff = (long long)blockIdx.y * ndof;
  PatchPos P = patch_pos(g, active ? pid : 0);
  if (active) {
    load_tile<T>(x + roff, g.N, P, lane, bufA);
    load_tile<T>(b + roff, g.N, P, lane, bufC);
    load_ext<T, 0>(t, x + roff, g.N, P, lane, ext);
  }
  __syncthreads();
  auto emit = [&](int, int base, int stride, const Line<T>& v) {
#pragma unroll
    for (int nu = 0; nu < n; ++nu) {
      T s = T(0);
#pragma unroll
      for (int p = 0; p < E; ++p) s += t->P[p * n + nu] * (bufC[base + p * stride] - scale * v.v[p]);
      bufA[base + nu * stride] = s;
    }
  };
  operator_passes<T>(t, bufA, bufB, ext, lane, active, emit);
  __syncthreads();
  // restrict along the remaining directions (y then x in 3-D; x in 2-D)
#pragma unroll
  for (int dir = D - 2; dir >= 0; --dir) {
    if (active) {
      // lines along dir whose coordinates in already-restricted directions are < n
      const int nlines = (D == 3) ? (dir == 1 ? E * n : n * n) : n;
      for (int i = lane; i < nlines; i += TPP) {
        int base, stride;
        if (D == 3) {
          if (dir == 1) { const int px = i % E, pz = i / E; base = px + pz * SZ; stride = SY; }
          else { const int py = i % n, pz = i / n; base = py * SY + pz * SZ; stride = 1; }
        } else { base = i * SY; stride = 1; }
        Line<T> v;
        load_line(bufA, base, stride, v);
#pragma unroll
        for (int nu = 0; nu < n; ++nu) {
          T s = T(0);
#pragma unroll
          for (int p = 0; p < E; ++p) s += t->P[p * n + nu] * v.v[p];
          bufA[base + nu * stride] = s;
        }
      }
    }
    __syncthreads();
  }
  if (active) {
    const int Nc = g.N / 2;
    const long long cell = cell_index(Nc, P.lo[0] / 2, P.lo[1] / 2, (D == 3) ? P.lo[2] / 2 : 0);
    T* out = bc + (long long)blockIdx.y * ndof_c + cell * NC;
    for (int i = lane; i < NC; i += TPP) {
      const int ax = i % n, ay = (i / n) % n, az = i / (n * n);
      out[i] = bufA[toff(ax, ay, az)];
    }
  }
}

// ------------------------------------------------- prolongation + add
template <typename T, int PPB>
__global__ void __launch_bounds__(TPP * PPB)
k_prolong(const Tab<K, T>* __restrict__ t, PatchGrid g, const T* __restrict__ xc,
          T* __restrict__ x, long long ndof, long long ndof_c) {
  __shared__ T smem[PPB * TS];
  const int slot = threadIdx.x / TPP, lane = threadIdx.x % TPP;
  const int pid = blockIdx.x * PPB + slot;
  const bool active = pid < g.npatch;
  T* tile = smem + slot * TS;
  PatchPos P = patch_pos(g, active ? pid : 0);
  if (active) {
    const int Nc = g.N / 2;
    const long long cell = cell_index(Nc, P.lo[0] / 2, P.lo[1] / 2, (D == 3) ? P.lo[2] / 2 : 0);
    const T* in = xc + (long long)blockIdx.y * ndof_c + cell * NC;
    for (int i = lane; i < NC; i += TPP) {
      const int ax = i % n, ay = (i / n) % n, az = i / (n * n);
      tile[toff(ax, ay, az)] = in[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int dir = 0; dir < D; ++dir) {
    if (active) {
      // lines along dir; coordinates in later directions still < n
      const int nlines = (D == 3) ? (dir == 0 ? n * n : dir == 1 ? E * n : E * E) : (dir == 0 ? n : E);
      for (int i = lane; i < nlines; i += TPP) {
        int base, stride;
        if (D == 3) {
          if (dir == 0) { const int py = i % n, pz = i / n; base = py * SY + pz * SZ; stride = 1; }
          else if (dir == 1) { const int px = i % E, pz = i / E; base = px + pz * SZ; stride = SY; }
          else { const int px = i % E, py = i / E; base = px + py * SY; stride = SZ; }
        } else {
          if (dir == 0) { base = i * SY; stride = 1; } else { base = i; stride = SY; }
        }
        T v[n];
#pragma unroll
        for (int nu = 0; nu < n; ++nu) v[nu] = tile[base + nu * stride];
#pragma unroll
        for (int p = 0; p < E; ++p) {
          T s = T(0);
#pragma unroll
          for (int nu = 0; nu < n; ++nu) s += t->P[p * n + nu] * v[nu];
          tile[base + p * stride] = s;
        }
      }
    }
    __syncthreads();
  }
  if (active) store_tile<T, true>(x + (long long)blockIdx.y * ndof, g.N, P, lane, tile);
}

// ---------------------------------------------------------- coarse solve
// Level 0 (N = 2): one patch, every node kept (type 3 in all directions).
template <typename T>
__global__ void __launch_bounds__(TPP)
k_coarse(const Tab<K, T>* __restrict__ t, T inv_scale, const T* __restrict__ b, T* __restrict__ x,
         long long ndof) {
  __shared__ T tile[TS];
  const int lane = threadIdx.x;
  PatchPos P;
#pragma unroll
  for (int i = 0; i < 3; ++i) { P.lo[i] = 0; P.ty[i] = 3; }
  const long long roff = (long long)blockIdx.y * ndof;
  load_tile<T>(b + roff, 2, P, lane, tile);
  __syncthreads();
  // S^T along z (3-D), y; then x with the eigenvalue scaling and S_x; then S_y, S_z
#pragma unroll
  for (int dir = D - 1; dir >= 1; --dir) {
    for (int i = lane; i < NL; i += TPP) {
      int base, stride;
      line_geom(dir, i, base, stride);
      Line<T> v, o;
      load_line(tile, base, stride, v);
      line_St_t<T, 3>(t, v, o);
      store_line(tile, base, stride, o);
    }
    __syncthreads();
  }
  for (int i = lane; i < NL; i += TPP) {
    int base, stride;
    line_geom(0, i, base, stride);
    const int qy = i % E, qz = i / E;
    T lt = t->lam[3][qy];
    if (D == 3) lt += t->lam[3][qz];
    Line<T> v, o;
    load_line(tile, base, stride, v);
    line_St_t<T, 3>(t, v, o);
#pragma unroll
    for (int q = 0; q < E; ++q) o.v[q] = o.v[q] * (inv_scale / (t->lam[3][q] + lt));
    line_S_t<T, 3>(t, o, v);
    store_line(tile, base, stride, v);
  }
  __syncthreads();
#pragma unroll
  for (int dir = 1; dir < D; ++dir) {
    for (int i = lane; i < NL; i += TPP) {
      int base, stride;
      line_geom(dir, i, base, stride);
      Line<T> v, o;
      load_line(tile, base, stride, v);
      line_S_t<T, 3>(t, v, o);
      store_line(tile, base, stride, o);
    }
    __syncthreads();
  }
  store_tile<T, false>(x + roff, 2, P, lane, tile);
}

// ------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_apply(const void* tab, PatchGrid g, T scale, const T* x, T* y, int nrhs,
                        long long ndof, hipStream_t s) {
  constexpr int PPB = PPB_DEFAULT;
  dim3 grid((g.npatch + PPB - 1) / PPB, nrhs);
  hipLaunchKernelGGL((k_apply<T, PPB>), grid, dim3(TPP * PPB), 0, s,
                     (const Tab<K, T>*)tab, g, scale, x, y, ndof);
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
template <typename T>
hipError_t launch_smooth(const void* tab, PatchGrid g, T scale, T inv_scale, int local_variant,
                         T* x, const T* b, int nrhs, long long ndof, hipStream_t s) {
  constexpr int PPB = PPB_DEFAULT;
  dim3 grid((g.npatch + PPB - 1) / PPB, nrhs);
  if (local_variant)
    hipLaunchKernelGGL((k_smooth<T, PPB, 2>), grid, dim3(TPP * PPB), 0, s,
                       (const Tab<K, T>*)tab, g, scale, inv_scale, x, b, ndof);
  else
    hipLaunchKernelGGL((k_smooth<T, PPB, 1>), grid, dim3(TPP * PPB), 0, s,
                       (const Tab<K, T>*)tab, g, scale, inv_scale, x, b, ndof);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_restrict(const void* tab, PatchGrid g, T scale, const T* x, const T* b, T* bc,
                           int nrhs, long long ndof, long long ndof_c, hipStream_t s) {
  constexpr int PPB = PPB_DEFAULT;
  dim3 grid((g.npatch + PPB - 1) / PPB, nrhs);
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

template <typename T>
KernelSet<T> make_set() {
  KernelSet<T> k;
  k.apply = &launch_apply<T>;
  k.mass = &launch_mass<T>;
  k.smooth = &launch_smooth<T>;
  k.restrict_residual = &launch_restrict<T>;
  k.prolongate_add = &launch_prolong<T>;
  k.coarse = &launch_coarse<T>;
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
