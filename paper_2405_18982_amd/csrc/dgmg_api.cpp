// C ABI of libdgmg.so (declared in include/dgmg.h): context, level
// hierarchy, host-orchestrated V-cycle and preconditioned CG.
//
// The V-cycle follows Sec. 3 with one kernel per operation, issued from the
// host in order on one stream (the paper's compute layout, Sec. 4.2):
//   level l = L .. 1: smooth (2^d colour launches), residual + restriction
//   level 0:          exact coarse solve
//   level l = 1 .. L: prolongation + add, smooth (colours reversed)
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dgmg.h"
#include "dgmg_blas.h"
#include "dgmg_internal.h"
#include "dgmg_scratch.h"
#include "dgmg_setup.h"

#define DGMG_API extern "C" __attribute__((visibility("default")))

DGMG_DECLARE_ENTRY(2, 1)
DGMG_DECLARE_ENTRY(2, 2)
DGMG_DECLARE_ENTRY(2, 3)
DGMG_DECLARE_ENTRY(2, 4)
DGMG_DECLARE_ENTRY(2, 5)
DGMG_DECLARE_ENTRY(2, 6)
DGMG_DECLARE_ENTRY(2, 7)
DGMG_DECLARE_ENTRY(3, 1)
DGMG_DECLARE_ENTRY(3, 2)
DGMG_DECLARE_ENTRY(3, 3)
DGMG_DECLARE_ENTRY(3, 4)
DGMG_DECLARE_ENTRY(3, 5)
DGMG_DECLARE_ENTRY(3, 6)
DGMG_DECLARE_ENTRY(3, 7)

namespace {

using dgmg::KernelEntry;
using dgmg::KernelSet;
using dgmg::PatchGrid;

const KernelEntry* kernels_for(int dim, int k) {
  static KernelEntry table[2][dgmg::kMaxDegree];
  static bool init = false;
  if (!init) {
    void (*f2[])(KernelEntry*) = {dgmg_kernels_d2_k1, dgmg_kernels_d2_k2, dgmg_kernels_d2_k3,
                                  dgmg_kernels_d2_k4, dgmg_kernels_d2_k5, dgmg_kernels_d2_k6,
                                  dgmg_kernels_d2_k7};
    void (*f3[])(KernelEntry*) = {dgmg_kernels_d3_k1, dgmg_kernels_d3_k2, dgmg_kernels_d3_k3,
                                  dgmg_kernels_d3_k4, dgmg_kernels_d3_k5, dgmg_kernels_d3_k6,
                                  dgmg_kernels_d3_k7};
    for (int i = 0; i < dgmg::kMaxDegree; ++i) {
      f2[i](&table[0][i]);
      f3[i](&table[1][i]);
    }
    init = true;
  }
  return &table[dim - 2][k - 1];
}

struct Level {
  int N = 0;
  long long ndof = 0;
  double h = 0;
  double* b64 = nullptr;
  double* x64 = nullptr;
  float* b32 = nullptr;
  float* x32 = nullptr;
  // second copy of x for the Full smoother (levels >= 1), one per precision
  double* alt64 = nullptr;
  float* alt32 = nullptr;
};

template <int K, typename T>
void fill_tab(int dim, const dgmg::HostTables& H, std::vector<unsigned char>& out) {
  using Tb = dgmg::Tab<K, T>;
  out.assign(sizeof(Tb), 0);
  Tb* t = reinterpret_cast<Tb*>(out.data());
  constexpr int E = 2 * (K + 1);
  // inverse eigenvalue sums, summed in the kernels' former order, in FP64
  const std::vector<double>* lams[3] = {H.lam, H.lamf, H.lamc};
  auto inv = [](double s) { return std::isinf(s) ? 0.0 : 1.0 / s; };
  for (int sp = 0; sp < 3; ++sp)
    for (int tx = 0; tx < 4; ++tx)
      for (int ty = 0; ty < 4; ++ty) {
        const std::vector<double>& lx = lams[sp][tx];
        const std::vector<double>& ly = lams[sp][ty];
        if (dim == 2) {
          T* r = t->rs[sp][tx * 4 + ty];
          for (int qy = 0; qy < E; ++qy)
            for (int qx = 0; qx < E; ++qx) r[qy * E + qx] = (T)inv(lx[qx] + ly[qy]);
          continue;
        }
        for (int tz = 0; tz < 4; ++tz) {
          const std::vector<double>& lz = lams[sp][tz];
          T* r = t->rs[sp][(tx * 4 + ty) * 4 + tz];
          for (int qz = 0; qz < E; ++qz)
            for (int qx = 0; qx < E; ++qx)
              for (int qy = 0; qy < E; ++qy) r[(qz * E + qx) * E + qy] = (T)inv(ly[qy] + (lx[qx] + lz[qz]));
        }
      }
  t->sigma = (T)H.sigma;
  for (int ty = 0; ty < 4; ++ty) {
    for (int i = 0; i < E * E; ++i) t->S[ty][i] = (T)H.S[ty][i];
    // unused eigenvalue slots: a huge finite value instead of +inf, so that the
    // kernels' reciprocal (estimate + Newton steps) returns ~0 without NaNs
    for (int i = 0; i < E; ++i)
      t->lam[ty][i] = std::isinf(H.lam[ty][i]) ? (T)(sizeof(T) == 8 ? 1e300 : 1e30) : (T)H.lam[ty][i];
    for (int i = 0; i < E * E; ++i) t->Sf[ty][i] = (T)H.Sf[ty][i];
    for (int i = 0; i < E; ++i) t->lamf[ty][i] = (T)H.lamf[ty][i];
    for (int i = 0; i < E * E; ++i) t->Sc[ty][i] = (T)H.Sc[ty][i];
    for (int i = 0; i < E; ++i)
      t->lamc[ty][i] = std::isinf(H.lamc[ty][i]) ? (T)(sizeof(T) == 8 ? 1e300 : 1e30) : (T)H.lamc[ty][i];
  }
}

template <typename T>
void fill_tab_k(int dim, int k, const dgmg::HostTables& H, std::vector<unsigned char>& out) {
  switch (k) {
    case 1: fill_tab<1, T>(dim, H, out); break;
    case 2: fill_tab<2, T>(dim, H, out); break;
    case 3: fill_tab<3, T>(dim, H, out); break;
    case 4: fill_tab<4, T>(dim, H, out); break;
    case 5: fill_tab<5, T>(dim, H, out); break;
    case 6: fill_tab<6, T>(dim, H, out); break;
    default: fill_tab<7, T>(dim, H, out); break;
  }
}

}  // namespace

struct dgmg_ctx {
  int dim = 0, k = 0, L = 0;
  double sigma = 0, kappa = 1;
  dgmg::HostTables host;
  const KernelEntry* ks = nullptr;
  std::vector<Level> lv;
  bool ready = false;
  int prec = 64, variant = 0, nrhs_max = 1;
  hipStream_t stream = nullptr;
  void* tab64 = nullptr;
  void* tab32 = nullptr;

  // Krylov workspace (finest level, FP64) and scalars
  double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double* scal = nullptr;  // kNumScal arrays of nrhs_max
  double *partial = nullptr, *partial2 = nullptr;
  int* active = nullptr;
  double* hbuf = nullptr;  // pinned host mirror of scalars
  int* hact = nullptr;
  // CG convergence decided on the device: norms of b (device, uploaded from
  // the pinned hnb once per solve), the check kernel's record (pinned host
  // memory, 4 doubles per right-hand side; rec_dev is its device address) and
  // the event the host waits on by polling
  double* nb = nullptr;
  double* hnb = nullptr;
  // coefficient gradient per right-hand side and in total (nrhs_max + 1)
  double* dk = nullptr;
  double* rec = nullptr;
  double* rec_dev = nullptr;
  hipEvent_t ev_check = nullptr;
  // V-cycle of the CG (r -> z) captured as a HIP graph, per nrhs; replayed on
  // the caller's stream.  Captured on the library's own stream (default
  // priority); invalidated when kappa changes.
  bool use_graph = true;
  // levels 1 and 0 of the V-cycle in one launch where the kernels allow it,
  // with two waves per patch where they allow that (DGMG_FUSE_BOTTOM at
  // set-up: 0 separate launches, 1 one wave per patch; to measure the effect)
  int fuse_bottom = 2;
  // workgroup shape and XCD-aware numbering of the tuned kernels, per
  // precision (0: FP64, 1: FP32); set by dgmg_autotune
  struct Tuning {
    int shape = 0;
    int remap = 1;
    double us = 0;
  };
  Tuning tune_apply[2];
  Tuning tune_smooth[2][dgmg::kMaxLevels];  // per precision and level
  hipStream_t cap_stream = nullptr;
  std::vector<hipGraphExec_t> vc_graph;  // index nrhs - 1
  // the FP32 V-cycle alone (finest-level b32 -> x32), for the CG with an
  // FP32 V-cycle, whose vector kernels convert on the fly
  std::vector<hipGraphExec_t> vc_graph32;
  // GMRES workspace (finest level, one right-hand side): Krylov basis V
  // (gm_cap + 1 vectors), preconditioned directions Z (gm_cap vectors),
  // device scalars and their pinned host mirror, partial sums
  double *gm_V = nullptr, *gm_Z = nullptr, *gm_s = nullptr, *gm_partial = nullptr;
  double* gm_h = nullptr;
  int gm_cap = 0;
  // device address of the library's scratch array on this context's device
  // (dgmg_vcycle_noalloc), looked up in dgmg_setup_levels
  void* scratch = nullptr;
  // The V-cycle's bottom levels 0..dense_lvl as a dense operator in the
  // V-cycle precision, built at set-up from the cycle from level dense_lvl
  // applied to unit vectors (row j = the operator's column j); applied with the scale dense_kappa / kappa (the V-cycle of kappa A_1
  // is that of A_1 divided by kappa) to at most kDenseMaxRhs right-hand
  // sides.  dense_part: the application's partial sums.
  int dense_lvl = -1;
  int dense_nd = 0;
  double* dense64 = nullptr;
  float* dense32 = nullptr;
  void* dense_part = nullptr;
  double dense_kappa = 1.0;
  bool use_dense = true;
  std::string err;
};

namespace {

enum { S_BB = 0, S_RR, S_PQ, S_ALPHA, S_RZ0, S_RZ1, S_ZQ, kNumScal };

dgmg_status fail(dgmg_ctx* c, dgmg_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, DGMG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define RET_IF(expr)                       \
  do {                                     \
    dgmg_status s_ = (expr);               \
    if (s_ != DGMG_OK) return s_;          \
  } while (0)

template <typename T>
T* dalloc(long long count, hipError_t& e) {
  void* p = nullptr;
  e = hipMalloc(&p, (size_t)count * sizeof(T));
  return e == hipSuccess ? (T*)p : nullptr;
}

// XCD-aware patch numbering: the tuned choice, unless DGMG_XCD_REMAP=0/1
// forces it (used to measure its effect).
int xcd_remap_flag(int tuned = 1) {
  static int env = -2;
  if (env == -2) {
    const char* e = std::getenv("DGMG_XCD_REMAP");
    env = (e && (e[0] == '0' || e[0] == '1')) ? (e[0] - '0') : -1;
  }
  return env >= 0 ? env : tuned;
}

PatchGrid grid_colour0(const dgmg_ctx* c, int N) {
  PatchGrid g{};
  g.N = N;
  g.xcd_remap = xcd_remap_flag();
  g.npatch = 1;
  for (int i = 0; i < 3; ++i) {
    g.cnt[i] = (i < c->dim) ? N / 2 : 1;
    g.off[i] = 0;
    g.npatch *= g.cnt[i];
  }
  return g;
}

// Patches of one colour: colour bit i = 0 takes the vertices v_i = 1, 3, ..,
// N - 1 (cells lo_i = 0, 2, .., N - 2), bit 1 the vertices 2, 4, .., N - 2.
// With `tiling` (Full smoother) bit 1 also takes the partial patches at
// lo_i = -1 and N - 1, so that the colour's patches cover every cell once.
PatchGrid grid_colour(const dgmg_ctx* c, int N, int colour, bool tiling = false) {
  PatchGrid g{};
  g.N = N;
  g.xcd_remap = xcd_remap_flag();
  g.npatch = 1;
  for (int i = 0; i < 3; ++i) {
    if (i < c->dim) {
      const int bit = (colour >> i) & 1;
      if (bit && tiling) {
        g.off[i] = -1;
        g.cnt[i] = N / 2 + 1;
      } else {
        g.off[i] = bit;
        g.cnt[i] = bit ? (N - 2) / 2 : N / 2;
      }
    } else {
      g.off[i] = 0;
      g.cnt[i] = 1;
    }
    g.npatch *= g.cnt[i];
  }
  return g;
}

double level_scale(const dgmg_ctx* c, int l) {
  return c->kappa * std::pow(c->lv[l].h, c->dim - 2);
}

template <typename T>
const KernelSet<T>& kset(const dgmg_ctx* c);
template <>
const KernelSet<double>& kset<double>(const dgmg_ctx* c) { return c->ks->f64; }
template <>
const KernelSet<float>& kset<float>(const dgmg_ctx* c) { return c->ks->f32; }
template <typename T>
void* tab_of(const dgmg_ctx* c) { return sizeof(T) == 8 ? c->tab64 : c->tab32; }
dgmg_status check_ready(dgmg_ctx* c) {
  if (!c) return DGMG_ERR_ARG;
  if (!c->ready) return fail(c, DGMG_ERR_STATE, "dgmg_setup_levels has not been called");
  return DGMG_OK;
}

dgmg_status check_level(dgmg_ctx* c, int level, int lo, int nrhs) {
  dgmg_status s = check_ready(c);
  if (s != DGMG_OK) return s;
  if (level < lo || level > c->L) return fail(c, DGMG_ERR_ARG, "level out of range");
  if (nrhs < 1 || nrhs > c->nrhs_max) return fail(c, DGMG_ERR_ARG, "nrhs out of range [1, nrhs_max]");
  return DGMG_OK;
}

// ------------------------------------------------------------ level ops
template <typename T>
constexpr int prec_index() { return sizeof(T) == 8 ? 0 : 1; }

template <typename T>
dgmg_status op_apply(dgmg_ctx* c, int l, const T* x, T* y, int nrhs) {
  const auto& tu = c->tune_apply[prec_index<T>()];
  PatchGrid g = grid_colour0(c, c->lv[l].N);
  g.xcd_remap = xcd_remap_flag(tu.remap);
  HIPCHK(c, kset<T>(c).apply[tu.shape](tab_of<T>(c), g, (T)level_scale(c, l), x, y, nrhs,
                                       c->lv[l].ndof, c->stream));
  return DGMG_OK;
}

// y = A_l(kappa = 1) x: the operator without the coefficient
dgmg_status op_apply_unit(dgmg_ctx* c, int l, const double* x, double* y, int nrhs) {
  const auto& tu = c->tune_apply[0];
  PatchGrid g = grid_colour0(c, c->lv[l].N);
  g.xcd_remap = xcd_remap_flag(tu.remap);
  const double sc = std::pow(c->lv[l].h, c->dim - 2);
  HIPCHK(c, kset<double>(c).apply[tu.shape](c->tab64, g, sc, x, y, nrhs, c->lv[l].ndof, c->stream));
  return DGMG_OK;
}

template <typename T>
T*& lvalt(Level& L);
template <>
double*& lvalt<double>(Level& L) { return L.alt64; }
template <>
float*& lvalt<float>(Level& L) { return L.alt32; }

template <typename T>
dgmg_status ensure_alt(dgmg_ctx* c);

// One smoothing step.  The Dirichlet kernels update x in place colour by
// colour.  The Full kernel alternates between x and the level's second copy:
// colour i reads one and writes the other, so after the 2^d colours (an even
// number) the result is back in x.  from_zero: the step starts from x = 0
// (pre-smoothing in the V-cycle); colour 0 then takes r = b and writes every
// node, so x need not be cleared first.
// alt: the second copy of x for the Full smoother (nullptr: the level's own).
template <typename T>
dgmg_status op_smooth(dgmg_ctx* c, int l, T* x, const T* b, int reverse, int nrhs,
                      bool from_zero = false, T* alt = nullptr) {
  const double sc = level_scale(c, l);
  const int nc = 1 << c->dim;
  const bool full = c->variant == DGMG_SMOOTH_FULL;
  T* cur = x;
  T* other = nullptr;
  if (full) {
    if (!alt) {
      RET_IF(ensure_alt<T>(c));
      alt = lvalt<T>(c->lv[l]);
    }
    other = alt;
  }
  for (int i = 0; i < nc; ++i) {
    const int col = reverse ? nc - 1 - i : i;
    PatchGrid g = grid_colour(c, c->lv[l].N, col, full);
    if (g.npatch == 0) continue;
    const auto& tu = c->tune_smooth[prec_index<T>()][l];
    g.xcd_remap = xcd_remap_flag(tu.remap);
    T* out = full ? other : cur;
    const int zero = (from_zero && !reverse && i == 0) ? 1 : 0;
    HIPCHK(c, kset<T>(c).smooth[tu.shape](tab_of<T>(c), g, (T)sc, (T)(1.0 / sc), c->variant, zero,
                                          cur, out, b, nrhs, c->lv[l].ndof, c->stream));
    if (full) {
      other = cur;
      cur = out;
    }
  }
  return DGMG_OK;
}

template <typename T>
dgmg_status op_restrict(dgmg_ctx* c, int l, const T* x, const T* b, T* bc, int nrhs) {
  HIPCHK(c, kset<T>(c).restrict_residual(tab_of<T>(c), grid_colour0(c, c->lv[l].N),
                                         (T)level_scale(c, l), x, b, bc, nrhs, c->lv[l].ndof,
                                         c->lv[l - 1].ndof, c->stream));
  return DGMG_OK;
}

template <typename T>
dgmg_status op_prolong(dgmg_ctx* c, int l, const T* xc, T* x, int nrhs) {
  HIPCHK(c, kset<T>(c).prolongate_add(tab_of<T>(c), grid_colour0(c, c->lv[l].N), xc, x, nrhs,
                                      c->lv[l].ndof, c->lv[l - 1].ndof, c->stream));
  return DGMG_OK;
}

template <typename T>
dgmg_status op_coarse(dgmg_ctx* c, const T* b, T* x, int nrhs) {
  HIPCHK(c, kset<T>(c).coarse(tab_of<T>(c), (T)(1.0 / level_scale(c, 0)), b, x, nrhs, c->lv[0].ndof,
                              c->stream));
  return DGMG_OK;
}

template <typename T>
dgmg_status zero_vec(dgmg_ctx* c, T* a, long long n) {
  if (sizeof(T) == 8) HIPCHK(c, dgmg::blas_zero_f64((double*)a, n, c->stream));
  else HIPCHK(c, dgmg::blas_zero_f32((float*)a, n, c->stream));
  return DGMG_OK;
}

template <typename T>
T*& lvb(Level& L);
template <>
double*& lvb<double>(Level& L) { return L.b64; }
template <>
float*& lvb<float>(Level& L) { return L.b32; }
template <typename T>
T*& lvx(Level& L);
template <>
double*& lvx<double>(Level& L) { return L.x64; }
template <>
float*& lvx<float>(Level& L) { return L.x32; }

// Second copies of x on levels 1..L for the Full smoother.
template <typename T>
dgmg_status ensure_alt(dgmg_ctx* c) {
  if (c->variant != DGMG_SMOOTH_FULL) return DGMG_OK;
  for (int l = 1; l <= c->L; ++l) {
    Level& L = c->lv[l];
    hipError_t e = hipSuccess;
    if (!lvalt<T>(L)) lvalt<T>(L) = dalloc<T>(L.ndof * c->nrhs_max, e);
    if (e != hipSuccess) return fail(c, DGMG_ERR_ALLOC, "level vector allocation failed");
  }
  return DGMG_OK;
}

// Library-owned level vectors of precision T on levels [0, upto].
template <typename T>
dgmg_status ensure_levels(dgmg_ctx* c, int upto) {
  for (int l = 0; l <= upto; ++l) {
    Level& L = c->lv[l];
    hipError_t e = hipSuccess;
    const long long cnt = L.ndof * c->nrhs_max;
    if (!lvb<T>(L)) lvb<T>(L) = dalloc<T>(cnt, e);
    if (e != hipSuccess) return fail(c, DGMG_ERR_ALLOC, "level vector allocation failed");
    if (!lvx<T>(L)) lvx<T>(L) = dalloc<T>(cnt, e);
    if (e != hipSuccess) return fail(c, DGMG_ERR_ALLOC, "level vector allocation failed");
  }
  return DGMG_OK;
}

#define RET(expr)                          \
  do {                                     \
    dgmg_status s_ = (expr);               \
    if (s_ != DGMG_OK) return s_;          \
  } while (0)

constexpr int kDenseMaxNd = 8192;  // largest bottom operator kept dense (537 MB in FP64)
// most right-hand sides per dense application (2..16 go through matrix-core
// tiles that read the matrix once); beyond that the bottom launch, which runs
// all of them side by side (one workgroup each) in about the time of one
constexpr int kDenseMaxRhs = 16;

template <typename T>
T* dense_of(const dgmg_ctx* c);
template <>
double* dense_of<double>(const dgmg_ctx* c) { return c->dense64; }
template <>
float* dense_of<float>(const dgmg_ctx* c) { return c->dense32; }

// Vectors of precision T on levels 0..L-1 (b, x) and the Full smoother's
// second copies on levels 1..L (alt), for one V-cycle.
template <typename T>
struct VBufs {
  T* b[dgmg::kMaxLevels] = {};
  T* x[dgmg::kMaxLevels] = {};
  T* alt[dgmg::kMaxLevels] = {};
};

// x = V(b) on level L with b, x given (may be caller or library buffers);
// coarser levels use the vectors of `bufs`, else the library's own of
// precision T.  top >= 0: the cycle from level top instead of L (b, x on
// that level).
template <typename T>
dgmg_status vcycle_T(dgmg_ctx* c, const T* bL, T* xL, int nrhs, const VBufs<T>* bufs = nullptr,
                     int top = -1) {
  if (!bufs) RET(ensure_levels<T>(c, c->L - 1));
  const int L = top < 0 ? c->L : top;
  auto Bw = [&](int l) -> T* { return bufs ? bufs->b[l] : lvb<T>(c->lv[l]); };
  auto B = [&](int l) -> const T* { return l == L ? bL : Bw(l); };
  auto X = [&](int l) -> T* { return l == L ? xL : (bufs ? bufs->x[l] : lvx<T>(c->lv[l])); };
  auto Alt = [&](int l) -> T* { return bufs ? bufs->alt[l] : nullptr; };
  // levels 1 and 0 (2-D: 2, 1 and 0) in one launch (same arithmetic as the
  // separate kernels), or levels 0..dense_lvl as one product with their
  // dense operator
  const bool fuse = c->fuse_bottom && kset<T>(c).bottom && c->variant != DGMG_SMOOTH_FULL;
  const bool fuse3 = fuse && c->fuse_bottom >= 2 && kset<T>(c).bottom3 && L >= 2;
  const bool dense = c->use_dense && dense_of<T>(c) && c->dense_lvl < L && nrhs <= kDenseMaxRhs;
  const int lo = dense ? c->dense_lvl + 1 : fuse3 ? 3 : fuse ? 2 : 1;
  for (int l = L; l >= lo; --l) {
    RET(op_smooth<T>(c, l, X(l), B(l), 0, nrhs, true, Alt(l)));
    RET(op_restrict<T>(c, l, X(l), B(l), Bw(l - 1), nrhs));
  }
  if (dense) {
    HIPCHK(c, dgmg::dense_apply<T>(dense_of<T>(c), c->dense_nd, B(lo - 1), X(lo - 1), nrhs,
                                   (T)(c->dense_kappa / c->kappa), (T*)c->dense_part, c->stream));
  } else if (fuse3) {
    const double s2 = level_scale(c, 2), s1 = level_scale(c, 1);
    HIPCHK(c, kset<T>(c).bottom3(tab_of<T>(c), c->variant, (T)s2, (T)(1.0 / s2), (T)s1, (T)(1.0 / s1),
                                 (T)(1.0 / level_scale(c, 0)), X(2), B(2), X(1), Bw(1), Bw(0), X(0),
                                 nrhs, c->lv[2].ndof, c->lv[1].ndof, c->lv[0].ndof, c->stream));
  } else if (fuse) {
    const double s1 = level_scale(c, 1);
    const int split = (c->fuse_bottom >= 2 && kset<T>(c).bottom_split) ? 1 : 0;
    HIPCHK(c, kset<T>(c).bottom(tab_of<T>(c), c->variant, split, (T)s1, (T)(1.0 / s1),
                                (T)(1.0 / level_scale(c, 0)), X(1), B(1), Bw(0), X(0), nrhs,
                                c->lv[1].ndof, c->lv[0].ndof, c->stream));
  } else {
    RET(op_coarse<T>(c, B(0), X(0), nrhs));
  }
  for (int l = lo; l <= L; ++l) {
    RET(op_prolong<T>(c, l, X(l - 1), X(l), nrhs));
    RET(op_smooth<T>(c, l, X(l), B(l), 1, nrhs, false, Alt(l)));
  }
  return DGMG_OK;
}

// Carve the vectors of one V-cycle of precision T for nrhs right-hand sides
// out of the scratch array (256-byte aligned pieces): b and x on levels
// 0..L-1, with `finest` also on level L (the FP32 V-cycle's input and output),
// and the Full smoother's second copies on levels 1..L.  Returns the bytes
// needed; fills `out` only if they fit in `cap`.
template <typename T>
size_t carve_scratch(const dgmg_ctx* c, int nrhs, bool finest, unsigned char* base, size_t cap,
                     VBufs<T>& out) {
  size_t used = 0;
  auto take = [&](long long count) -> T* {
    const size_t bytes = ((size_t)count * sizeof(T) + 255) & ~size_t(255);
    T* p = (used + bytes <= cap) ? (T*)(base + used) : nullptr;
    used += bytes;
    return p;
  };
  const int top = finest ? c->L : c->L - 1;
  for (int l = 0; l <= top; ++l) {
    out.b[l] = take(c->lv[l].ndof * nrhs);
    out.x[l] = take(c->lv[l].ndof * nrhs);
  }
  if (c->variant == DGMG_SMOOTH_FULL)
    for (int l = 1; l <= c->L; ++l) out.alt[l] = take(c->lv[l].ndof * nrhs);
  return used;
}

// z = V(r) in the context precision (FP64 vectors in and out).
dgmg_status precondition(dgmg_ctx* c, const double* r, double* z, int nrhs) {
  if (c->prec == 64) return vcycle_T<double>(c, r, z, nrhs);
  RET(ensure_levels<float>(c, c->L));
  Level& T = c->lv[c->L];
  const long long n = T.ndof * nrhs;
  HIPCHK(c, dgmg::blas_f64_to_f32(r, T.b32, n, c->stream));
  RET(vcycle_T<float>(c, T.b32, T.x32, nrhs));
  HIPCHK(c, dgmg::blas_f32_to_f64(T.x32, z, n, c->stream));
  return DGMG_OK;
}

// The bottom levels of the V-cycle as a dense operator (see dgmg_ctx): the
// cycle from level m (the finest level below L with at most kDenseMaxNd
// DoFs), applied to the nd unit vectors of level m, gives the operator's
// columns (the Full smoother with second copies of x on levels 1..m).  An
// allocation failure leaves the context without it (the kernels stay in use).
template <typename T>
dgmg_status build_dense(dgmg_ctx* c) {
  int m = 0;
  for (int l = 1; l < c->L; ++l)
    if (c->lv[l].ndof <= kDenseMaxNd) m = l;
  if (m == 0) return DGMG_OK;
  const int nd = (int)c->lv[m].ndof;
  hipError_t e = hipSuccess;
  std::vector<void*> tmp;
  auto alloc = [&](long long count) -> T* {
    if (e != hipSuccess) return nullptr;
    T* p = dalloc<T>(count, e);
    if (p) tmp.push_back(p);
    return p;
  };
  auto release = [&]() {
    for (void* p : tmp) hipFree(p);
    tmp.clear();
  };
  T* Xm = alloc((long long)nd * nd);
  T* Bm = alloc((long long)nd * nd);
  VBufs<T> bufs;
  for (int l = 0; l < m; ++l) {
    bufs.b[l] = alloc(c->lv[l].ndof * nd);
    bufs.x[l] = alloc(c->lv[l].ndof * nd);
  }
  if (c->variant == DGMG_SMOOTH_FULL)
    for (int l = 1; l <= m; ++l) bufs.alt[l] = alloc(c->lv[l].ndof * nd);
  T* part = alloc((long long)dgmg::kDenseChunks * kDenseMaxRhs * nd);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release();
    return DGMG_OK;
  }
  dgmg_status st = DGMG_OK;
  e = dgmg::unit_batch<T>(Bm, nd, 0, nd, c->stream);
  if (e == hipSuccess) st = vcycle_T<T>(c, Bm, Xm, nd, &bufs, m);
  if (e == hipSuccess && st == DGMG_OK) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess || st != DGMG_OK) {
    (void)hipStreamSynchronize(c->stream);
    release();
    if (st != DGMG_OK) return st;
    return fail(c, DGMG_ERR_HIP, std::string("dense bottom set-up: ") + hipGetErrorString(e));
  }
  // keep the operator and the partial sums, free the rest
  for (void* p : tmp)
    if (p != Xm && p != part) hipFree(p);
  tmp.clear();
  if (sizeof(T) == 8) c->dense64 = (double*)Xm;
  else c->dense32 = (float*)Xm;
  c->dense_part = part;
  c->dense_lvl = m;
  c->dense_nd = nd;
  c->dense_kappa = c->kappa;
  return DGMG_OK;
}

void drop_graphs(dgmg_ctx* c) {
  for (auto* v : {&c->vc_graph, &c->vc_graph32})
    for (hipGraphExec_t& g : *v)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
}

// Wait for an event by polling it (no sleep on the stream: the host sees the
// completion within microseconds and launches the next work at once).
dgmg_status poll_event(dgmg_ctx* c, hipEvent_t ev) {
  for (;;) {
    const hipError_t e = hipEventQuery(ev);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) return fail(c, DGMG_ERR_HIP, std::string("event: ") + hipGetErrorString(e));
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return DGMG_OK;
}

// z = V(r) for the CG: replay (capturing on first use) the graph of the
// V-cycle on the CG workspace for this nrhs.  raw32 (FP32 V-cycle only): the
// V-cycle alone from the finest level's b32 to its x32, the conversions left
// to the CG's vector kernels.
dgmg_status precondition_cg(dgmg_ctx* c, int nrhs, bool raw32 = false) {
  auto body = [&]() -> dgmg_status {
    if (!raw32) return precondition(c, c->r, c->z, nrhs);
    Level& T = c->lv[c->L];
    return vcycle_T<float>(c, T.b32, T.x32, nrhs);
  };
  if (!c->use_graph) return body();
  auto& cache = raw32 ? c->vc_graph32 : c->vc_graph;
  if ((int)cache.size() < c->nrhs_max) cache.resize(c->nrhs_max, nullptr);
  hipGraphExec_t& ex = cache[nrhs - 1];
  if (!ex) {
    if (!c->cap_stream) HIPCHK(c, hipStreamCreate(&c->cap_stream));
    // level buffers must exist before capture (allocation is not capturable)
    if (c->prec == 64) RET(ensure_levels<double>(c, c->L - 1));
    else RET(ensure_levels<float>(c, c->L));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipStream_t user = c->stream;
    c->stream = c->cap_stream;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    dgmg_status st = DGMG_OK;
    if (e == hipSuccess) st = body();
    hipError_t e2 = (e == hipSuccess) ? hipStreamEndCapture(c->cap_stream, &graph) : e;
    c->stream = user;
    if (st != DGMG_OK) {
      if (graph) hipGraphDestroy(graph);
      return st;
    }
    if (e2 != hipSuccess) return fail(c, DGMG_ERR_HIP, std::string("V-cycle capture: ") + hipGetErrorString(e2));
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
      ex = nullptr;
      return fail(c, DGMG_ERR_HIP, std::string("V-cycle graph instantiate: ") + hipGetErrorString(e));
    }
  }
  HIPCHK(c, hipGraphLaunch(ex, c->stream));
  return DGMG_OK;
}

}  // namespace

// ================================================================ C ABI

DGMG_API dgmg_status dgmg_setup_mesh(int dim, int degree, int finest_level, double penalty_sigma,
                                     double kappa, dgmg_ctx** out) {
  if (!out) return DGMG_ERR_ARG;
  *out = nullptr;
  if (dim != 2 && dim != 3) return DGMG_ERR_ARG;
  if (degree < 1 || degree > dgmg::kMaxDegree) return DGMG_ERR_ARG;
  if (finest_level < 1 || finest_level > 20) return DGMG_ERR_ARG;
  if (!(penalty_sigma > 0) || !std::isfinite(penalty_sigma)) return DGMG_ERR_ARG;
  if (!(kappa > 0) || !std::isfinite(kappa)) return DGMG_ERR_ARG;
  const double nd = std::pow(2.0, (finest_level + 1) * dim) * std::pow(degree + 1.0, dim);
  if (nd >= std::pow(2.0, 40)) return DGMG_ERR_ARG;
  dgmg_ctx* c = new (std::nothrow) dgmg_ctx;
  if (!c) return DGMG_ERR_ALLOC;
  c->dim = dim;
  c->k = degree;
  c->L = finest_level;
  c->sigma = penalty_sigma;
  c->kappa = kappa;
  const char* err = nullptr;
  if (!dgmg::build_host_tables(degree, penalty_sigma, c->host, &err)) {
    delete c;
    return DGMG_ERR_ARG;
  }
  c->lv.resize(finest_level + 1);
  for (int l = 0; l <= finest_level; ++l) {
    Level& L = c->lv[l];
    L.N = 1 << (l + 1);
    L.h = 1.0 / L.N;
    L.ndof = 1;
    for (int i = 0; i < dim; ++i) L.ndof *= (long long)L.N * (degree + 1);
  }
  c->ks = kernels_for(dim, degree);
  *out = c;
  return DGMG_OK;
}

DGMG_API dgmg_status dgmg_setup_levels(dgmg_ctx* c, int vcycle_precision, int smoother_variant,
                                       int nrhs_max, void* hip_stream) {
  if (!c) return DGMG_ERR_ARG;
  if (c->ready) return fail(c, DGMG_ERR_STATE, "levels already set up");
  if (vcycle_precision != DGMG_FP64 && vcycle_precision != DGMG_FP32)
    return fail(c, DGMG_ERR_ARG, "vcycle_precision must be 64 or 32");
  if (smoother_variant != DGMG_SMOOTH_EXACT && smoother_variant != DGMG_SMOOTH_LOCAL &&
      smoother_variant != DGMG_SMOOTH_FULL && smoother_variant != DGMG_SMOOTH_CLAMPED)
    return fail(c, DGMG_ERR_ARG, "unknown smoother variant");
  if (smoother_variant == DGMG_SMOOTH_CLAMPED && c->k < 3)
    return fail(c, DGMG_ERR_ARG, "the clamped kernel needs degree >= 3");
  if (nrhs_max < 1 || nrhs_max > 4096) return fail(c, DGMG_ERR_ARG, "nrhs_max out of range");
  c->prec = vcycle_precision;
  c->variant = smoother_variant;
  {
    const char* e = std::getenv("DGMG_FUSE_BOTTOM");
    c->fuse_bottom = (e && e[0] == '0') ? 0 : (e && e[0] == '1') ? 1 : 2;
  }
  c->nrhs_max = nrhs_max;
  c->stream = (hipStream_t)hip_stream;
  // untuned apply: face data in registers where the kernels have it (the
  // autotuner may still choose another shape for the FP64 apply)
  c->tune_apply[0].shape = kset<double>(c).apply_rf ? 2 : 0;
  c->tune_apply[1].shape = kset<float>(c).apply_rf ? 2 : 0;
  std::vector<unsigned char> t64, t32;
  fill_tab_k<double>(c->dim, c->k, c->host, t64);
  fill_tab_k<float>(c->dim, c->k, c->host, t32);
  HIPCHK(c, hipMalloc(&c->tab64, t64.size()));
  HIPCHK(c, hipMalloc(&c->tab32, t32.size()));
  HIPCHK(c, hipMemcpy(c->tab64, t64.data(), t64.size(), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->tab32, t32.data(), t32.size(), hipMemcpyHostToDevice));
  const long long nL = c->lv[c->L].ndof * nrhs_max;
  hipError_t e = hipSuccess;
  c->r = dalloc<double>(nL, e);
  if (e == hipSuccess) c->z = dalloc<double>(nL, e);
  if (e == hipSuccess) c->p = dalloc<double>(nL, e);
  if (e == hipSuccess) c->q = dalloc<double>(nL, e);
  if (e == hipSuccess) c->scal = dalloc<double>((long long)kNumScal * nrhs_max, e);
  if (e == hipSuccess) c->partial = dalloc<double>((long long)dgmg::kRedBlocks * nrhs_max, e);
  if (e == hipSuccess) c->partial2 = dalloc<double>((long long)dgmg::kRedBlocks * nrhs_max, e);
  if (e == hipSuccess) c->active = dalloc<int>(nrhs_max, e);
  if (e == hipSuccess) c->nb = dalloc<double>(nrhs_max, e);
  if (e == hipSuccess) c->dk = dalloc<double>(nrhs_max + 1, e);
  if (e != hipSuccess) return fail(c, DGMG_ERR_ALLOC, "workspace allocation failed");
  HIPCHK(c, hipHostMalloc((void**)&c->hbuf, sizeof(double) * kNumScal * nrhs_max));
  HIPCHK(c, hipHostMalloc((void**)&c->hact, sizeof(int) * nrhs_max));
  HIPCHK(c, hipHostMalloc((void**)&c->hnb, sizeof(double) * nrhs_max));
  HIPCHK(c, hipHostMalloc((void**)&c->rec, sizeof(double) * 4 * nrhs_max));
  HIPCHK(c, hipHostGetDevicePointer((void**)&c->rec_dev, c->rec, 0));
  HIPCHK(c, hipEventCreateWithFlags(&c->ev_check, hipEventDisableTiming));
  HIPCHK(c, dgmg::scratch_address(&c->scratch));
  c->ready = true;
  if (vcycle_precision == DGMG_FP64) RET(ensure_levels<double>(c, c->L - 1));
  else RET(ensure_levels<float>(c, c->L));
  RET(ensure_alt<double>(c));
  if (vcycle_precision == DGMG_FP32) RET(ensure_alt<float>(c));
  if (vcycle_precision == DGMG_FP64) RET(build_dense<double>(c));
  else RET(build_dense<float>(c));
  return DGMG_OK;
}

DGMG_API dgmg_status dgmg_set_stream(dgmg_ctx* c, void* hip_stream) {
  if (!c) return DGMG_ERR_ARG;
  c->stream = (hipStream_t)hip_stream;
  return DGMG_OK;
}

DGMG_API dgmg_status dgmg_use_graphs(dgmg_ctx* c, int enable) {
  if (!c) return DGMG_ERR_ARG;
  c->use_graph = enable != 0;
  if (!c->use_graph) drop_graphs(c);
  return DGMG_OK;
}

DGMG_API dgmg_status dgmg_use_dense_bottom(dgmg_ctx* c, int enable) {
  if (!c) return DGMG_ERR_ARG;
  c->use_dense = enable != 0;
  drop_graphs(c);  // graphs hold the previous bottom
  return DGMG_OK;
}

DGMG_API int dgmg_dense_bottom_level(const dgmg_ctx* c) {
  if (!c) return -1;
  return (c->prec == 64 ? c->dense64 != nullptr : c->dense32 != nullptr) ? c->dense_lvl : -1;
}

DGMG_API dgmg_status dgmg_set_kappa(dgmg_ctx* c, double kappa) {
  if (!c) return DGMG_ERR_ARG;
  if (!(kappa > 0) || !std::isfinite(kappa)) return fail(c, DGMG_ERR_ARG, "kappa must be positive");
  if (kappa != c->kappa) drop_graphs(c);  // level scales are baked into the graphs
  c->kappa = kappa;
  return DGMG_OK;
}

DGMG_API long long dgmg_level_ndofs(const dgmg_ctx* c, int level) {
  if (!c || level < 0 || level > c->L) return -1;
  return c->lv[level].ndof;
}

DGMG_API int dgmg_level_cells(const dgmg_ctx* c, int level) {
  if (!c || level < 0 || level > c->L) return -1;
  return c->lv[level].N;
}

DGMG_API int dgmg_finest_level(const dgmg_ctx* c) { return c ? c->L : -1; }

DGMG_API dgmg_status dgmg_node_coords(const dgmg_ctx* c, int level, double* xyz) {
  if (!c || !xyz || level < 0 || level > c->L) return DGMG_ERR_ARG;
  const int N = c->lv[level].N, n = c->k + 1, d = c->dim;
  const double h = c->lv[level].h;
  const long long ncell = (long long)std::pow((double)N, d);
  const int nc = (int)std::pow((double)n, d);
  long long idx = 0;
  for (long long cell = 0; cell < ncell; ++cell) {
    const long long cc[3] = {cell % N, (cell / N) % N, cell / ((long long)N * N)};
    for (int loc = 0; loc < nc; ++loc) {
      const int a[3] = {loc % n, (loc / n) % n, loc / (n * n)};
      for (int i = 0; i < d; ++i) xyz[idx * d + i] = (cc[i] + c->host.nodes[a[i]]) * h;
      ++idx;
    }
  }
  return DGMG_OK;
}

DGMG_API dgmg_status dgmg_apply_sipg(dgmg_ctx* c, int level, const double* x, double* y, int nrhs) {
  RET(check_level(c, level, 0, nrhs));
  if (!x || !y) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_apply<double>(c, level, x, y, nrhs);
}

DGMG_API dgmg_status dgmg_apply_sipg_f32(dgmg_ctx* c, int level, const float* x, float* y, int nrhs) {
  RET(check_level(c, level, 0, nrhs));
  if (!x || !y) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_apply<float>(c, level, x, y, nrhs);
}

DGMG_API dgmg_status dgmg_apply_mass(dgmg_ctx* c, int level, const double* x, double* y, int nrhs) {
  RET(check_level(c, level, 0, nrhs));
  if (!x || !y) return fail(c, DGMG_ERR_ARG, "null vector");
  const double sc = std::pow(c->lv[level].h, c->dim);
  HIPCHK(c, c->ks->f64.mass(c->tab64, grid_colour0(c, c->lv[level].N), sc, x, y, nrhs,
                            c->lv[level].ndof, c->stream));
  return DGMG_OK;
}

DGMG_API dgmg_status dgmg_smooth_patch(dgmg_ctx* c, int level, double* x, const double* b,
                                       int reverse_colours, int nrhs) {
  RET(check_level(c, level, 1, nrhs));
  if (!x || !b) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_smooth<double>(c, level, x, b, reverse_colours, nrhs);
}

DGMG_API dgmg_status dgmg_smooth_patch_f32(dgmg_ctx* c, int level, float* x, const float* b,
                                           int reverse_colours, int nrhs) {
  RET(check_level(c, level, 1, nrhs));
  if (!x || !b) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_smooth<float>(c, level, x, b, reverse_colours, nrhs);
}

DGMG_API dgmg_status dgmg_restrict_residual(dgmg_ctx* c, int level, const double* x,
                                            const double* b, double* bc, int nrhs) {
  RET(check_level(c, level, 1, nrhs));
  if (!x || !b || !bc) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_restrict<double>(c, level, x, b, bc, nrhs);
}

DGMG_API dgmg_status dgmg_restrict_residual_f32(dgmg_ctx* c, int level, const float* x,
                                                const float* b, float* bc, int nrhs) {
  RET(check_level(c, level, 1, nrhs));
  if (!x || !b || !bc) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_restrict<float>(c, level, x, b, bc, nrhs);
}

DGMG_API dgmg_status dgmg_prolongate_add(dgmg_ctx* c, int level, const double* xc, double* x,
                                         int nrhs) {
  RET(check_level(c, level, 1, nrhs));
  if (!x || !xc) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_prolong<double>(c, level, xc, x, nrhs);
}

DGMG_API dgmg_status dgmg_prolongate_add_f32(dgmg_ctx* c, int level, const float* xc, float* x,
                                             int nrhs) {
  RET(check_level(c, level, 1, nrhs));
  if (!x || !xc) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_prolong<float>(c, level, xc, x, nrhs);
}

DGMG_API dgmg_status dgmg_coarse_solve(dgmg_ctx* c, const double* b, double* x, int nrhs) {
  RET(check_level(c, 0, 0, nrhs));
  if (!x || !b) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_coarse<double>(c, b, x, nrhs);
}

DGMG_API dgmg_status dgmg_coarse_solve_f32(dgmg_ctx* c, const float* b, float* x, int nrhs) {
  RET(check_level(c, 0, 0, nrhs));
  if (!x || !b) return fail(c, DGMG_ERR_ARG, "null vector");
  return op_coarse<float>(c, b, x, nrhs);
}

DGMG_API dgmg_status dgmg_vcycle(dgmg_ctx* c, const double* b, double* x, int nrhs) {
  RET(check_level(c, c ? c->L : 0, 0, nrhs));
  if (!x || !b) return fail(c, DGMG_ERR_ARG, "null vector");
  return precondition(c, b, x, nrhs);
}

// dgmg_vcycle with the coarse-level vectors (and, for an FP32 V-cycle, the
// finest level's FP32 copies; for the Full smoother, the second copies of x)
// in the library's per-device scratch array instead of the context's own
// vectors; no graph, no allocation.  Shares the kernels of dgmg_vcycle.
DGMG_API dgmg_status dgmg_vcycle_noalloc(dgmg_ctx* c, const double* b, double* x, int nrhs) {
  RET(check_level(c, c ? c->L : 0, 0, nrhs));
  if (!x || !b) return fail(c, DGMG_ERR_ARG, "null vector");
  if (!c->scratch) return fail(c, DGMG_ERR_STATE, "scratch array address not available");
  unsigned char* base = (unsigned char*)c->scratch;
  char msg[160];
  if (c->prec == 64) {
    VBufs<double> bufs;
    const size_t need = carve_scratch<double>(c, nrhs, false, base, dgmg::kScratchBytes, bufs);
    if (need > dgmg::kScratchBytes) {
      std::snprintf(msg, sizeof msg, "vcycle_noalloc needs %zu bytes of scratch, the maximum is %zu",
                    need, dgmg::kScratchBytes);
      return fail(c, DGMG_ERR_ARG, msg);
    }
    return vcycle_T<double>(c, b, x, nrhs, &bufs);
  }
  VBufs<float> bufs;
  const size_t need = carve_scratch<float>(c, nrhs, true, base, dgmg::kScratchBytes, bufs);
  if (need > dgmg::kScratchBytes) {
    std::snprintf(msg, sizeof msg, "vcycle_noalloc needs %zu bytes of scratch, the maximum is %zu",
                  need, dgmg::kScratchBytes);
    return fail(c, DGMG_ERR_ARG, msg);
  }
  const int L = c->L;
  const long long n = c->lv[L].ndof * nrhs;
  HIPCHK(c, dgmg::blas_f64_to_f32(b, bufs.b[L], n, c->stream));
  RET(vcycle_T<float>(c, bufs.b[L], bufs.x[L], nrhs, &bufs));
  HIPCHK(c, dgmg::blas_f32_to_f64(bufs.x[L], x, n, c->stream));
  return DGMG_OK;
}

DGMG_API dgmg_status dgmg_vcycle_f32(dgmg_ctx* c, const float* b, float* x, int nrhs) {
  RET(check_level(c, c ? c->L : 0, 0, nrhs));
  if (!x || !b) return fail(c, DGMG_ERR_ARG, "null vector");
  return vcycle_T<float>(c, b, x, nrhs);
}

DGMG_API dgmg_status dgmg_pcg_solve(dgmg_ctx* c, const double* b, double* x, int use_initial_guess,
                                    double rtol, int maxit, int nrhs, int* iters, double* relres) {
  RET(check_level(c, c ? c->L : 0, 0, nrhs));
  if (!x || !b || !iters || !relres) return fail(c, DGMG_ERR_ARG, "null argument");
  if (!(rtol > 0) || maxit < 1) return fail(c, DGMG_ERR_ARG, "rtol must be > 0 and maxit >= 1");
  const long long n = c->lv[c->L].ndof;
  hipStream_t s = c->stream;
  const int R = c->nrhs_max;
  double* bb = c->scal + S_BB * R;
  double* rr = c->scal + S_RR * R;
  double* pq = c->scal + S_PQ * R;
  double* alpha = c->scal + S_ALPHA * R;
  double* rzb[2] = {c->scal + S_RZ0 * R, c->scal + S_RZ1 * R};
  double* zq = c->scal + S_ZQ * R;
  const int flexible = (c->prec == 32);
  // r = b - A x (or b), |b|^2
  if (use_initial_guess) {
    RET(op_apply<double>(c, c->L, x, c->q, nrhs));
    HIPCHK(c, dgmg::blas_sub(b, c->q, c->r, n * nrhs, s));
  } else {
    RET(zero_vec<double>(c, x, n * nrhs));
    HIPCHK(c, hipMemcpyAsync(c->r, b, sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(c, dgmg::blas_dot2(b, b, c->r, c->r, n, nrhs, c->partial, c->partial2, bb, rr, s));
  HIPCHK(c, hipMemcpyAsync(c->hbuf, c->scal, sizeof(double) * 2 * R, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  std::vector<double> nb(nrhs);
  bool any = false;
  for (int j = 0; j < nrhs; ++j) {
    const double b2 = c->hbuf[S_BB * R + j], r2 = c->hbuf[S_RR * R + j];
    if (!std::isfinite(b2) || !std::isfinite(r2))
      return fail(c, DGMG_ERR_ARG, "right-hand side or initial guess contains NaN/Inf");
    nb[j] = std::sqrt(b2);
    iters[j] = 0;
    relres[j] = (b2 > 0) ? std::sqrt(r2) / nb[j] : 0.0;
    c->hact[j] = (b2 > 0 && relres[j] > rtol) ? 1 : 0;
    any = any || c->hact[j];
  }
  if (!any) return DGMG_OK;
  for (int j = 0; j < nrhs; ++j) c->hnb[j] = nb[j];
  HIPCHK(c, hipMemcpyAsync(c->nb, c->hnb, sizeof(double) * nrhs, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->active, c->hact, sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
  // FP32 V-cycle: it runs from the finest level's b32 to its x32 and the
  // vector kernels convert on the way (the update of x and r writes
  // b32 = (float) r, the dot products and the update of p read z = x32 in
  // FP64), the same values as converting whole vectors around the V-cycle
  float* b32 = nullptr;
  const float* z32 = nullptr;
  if (flexible) {
    RET(ensure_levels<float>(c, c->L));
    b32 = c->lv[c->L].b32;
    z32 = c->lv[c->L].x32;
    HIPCHK(c, dgmg::blas_f64_to_f32(c->r, b32, n * nrhs, s));
    RET(precondition_cg(c, nrhs, true));
    HIPCHK(c, dgmg::blas_dot2_z32(c->r, z32, nullptr, nullptr, n, nrhs, c->partial, nullptr, s));
    HIPCHK(c, dgmg::blas_finalize(c->partial, n, nrhs, rzb[0], s));
    HIPCHK(c, dgmg::blas_f32_to_f64(z32, c->p, n * nrhs, s));
  } else {
    RET(precondition_cg(c, nrhs));
    HIPCHK(c, dgmg::blas_dot2(c->r, c->z, nullptr, nullptr, n, nrhs, c->partial, nullptr, rzb[0],
                              nullptr, s));
    HIPCHK(c, hipMemcpyAsync(c->p, c->z, sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, s));
  }
  dgmg_status status = DGMG_ERR_NOT_CONVERGED;
  for (int it = 1; it <= maxit; ++it) {
    double* rz_old = rzb[(it - 1) & 1];
    double* rz_new = rzb[it & 1];
    RET(op_apply<double>(c, c->L, c->p, c->q, nrhs));
    // p^T q stays as first-stage partial sums; the update finishes it
    HIPCHK(c, dgmg::blas_dot2(c->p, c->q, nullptr, nullptr, n, nrhs, c->partial, nullptr, nullptr,
                              nullptr, s));
    // the check kernel decides convergence on the device (active mask for the
    // next iteration) and records (|r|^2, p^T q, relres, active) in pinned
    // host memory; the host polls the event instead of sleeping on the stream
    HIPCHK(c, dgmg::blas_update_xr(x, c->r, c->p, c->q, rz_old, c->partial, pq, c->active, n, nrhs,
                                   alpha, c->partial2, b32, s));
    HIPCHK(c, dgmg::blas_cg_check(c->partial2, n, nrhs, rr, pq, c->nb, rtol, c->active, c->rec_dev, s));
    HIPCHK(c, hipEventRecord(c->ev_check, s));
    RET(poll_event(c, c->ev_check));
    any = false;
    for (int j = 0; j < nrhs; ++j) {
      if (!c->hact[j]) continue;
      const double r2 = c->rec[4 * j + 0], p2 = c->rec[4 * j + 1];
      if (!(p2 > 0) || !std::isfinite(p2) || !std::isfinite(r2))
        return fail(c, DGMG_ERR_BREAKDOWN, "CG breakdown: p^T A p <= 0 or non-finite scalar");
      iters[j] = it;
      relres[j] = c->rec[4 * j + 2];
      c->hact[j] = c->rec[4 * j + 3] != 0.0 ? 1 : 0;
      any = any || c->hact[j];
    }
    if (!any) { status = DGMG_OK; break; }
    RET(precondition_cg(c, nrhs, flexible));
    // r^T z (and z^T q) stay as partial sums; the update of p finishes them
    if (flexible) {
      HIPCHK(c, dgmg::blas_dot2_z32(c->r, z32, z32, c->q, n, nrhs, c->partial, c->partial2, s));
      HIPCHK(c, dgmg::blas_update_p_z32(c->p, z32, c->partial, c->partial2, rz_new, zq, rz_old, alpha,
                                        c->active, 1, n, nrhs, s));
    } else {
      HIPCHK(c, dgmg::blas_dot2(c->r, c->z, nullptr, nullptr, n, nrhs, c->partial, c->partial2,
                                nullptr, nullptr, s));
      HIPCHK(c, dgmg::blas_update_p(c->p, c->z, c->partial, c->partial2, rz_new, zq, rz_old, alpha,
                                    c->active, 0, n, nrhs, s));
    }
  }
  HIPCHK(c, hipStreamSynchronize(s));
  if (status != DGMG_OK) c->err = "maximum number of iterations reached";
  return status;
}

namespace {

void free_gmres(dgmg_ctx* c) {
  hipFree(c->gm_V);
  hipFree(c->gm_Z);
  hipFree(c->gm_s);
  hipFree(c->gm_partial);
  if (c->gm_h) hipHostFree(c->gm_h);
  c->gm_V = c->gm_Z = c->gm_s = c->gm_partial = c->gm_h = nullptr;
  c->gm_cap = 0;
}

// Grow the GMRES workspace to cap steps, keeping the first keepV basis
// vectors and keepZ directions (the basis grows with the iteration, so a
// large maxit costs memory only when the iteration actually runs that long).
dgmg_status ensure_gmres(dgmg_ctx* c, int cap, int keepV, int keepZ) {
  if (cap <= c->gm_cap) return DGMG_OK;
  const long long n = c->lv[c->L].ndof;
  hipError_t e = hipSuccess;
  double* V = dalloc<double>((long long)(cap + 1) * n, e);
  double* Z = (e == hipSuccess) ? dalloc<double>((long long)cap * n, e) : nullptr;
  double* sc = (e == hipSuccess) ? dalloc<double>(3LL * (cap + 2), e) : nullptr;
  double* part = (e == hipSuccess) ? dalloc<double>((long long)(cap + 1) * dgmg::kRedBlocks, e) : nullptr;
  double* hh = nullptr;
  if (e == hipSuccess) e = hipHostMalloc((void**)&hh, sizeof(double) * 3 * (cap + 2));
  if (e != hipSuccess) {
    hipFree(V);
    hipFree(Z);
    hipFree(sc);
    hipFree(part);
    return fail(c, DGMG_ERR_ALLOC, "GMRES workspace allocation failed");
  }
  if (keepV > 0)
    HIPCHK(c, hipMemcpyAsync(V, c->gm_V, sizeof(double) * n * keepV, hipMemcpyDeviceToDevice, c->stream));
  if (keepZ > 0)
    HIPCHK(c, hipMemcpyAsync(Z, c->gm_Z, sizeof(double) * n * keepZ, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  free_gmres(c);
  c->gm_V = V;
  c->gm_Z = Z;
  c->gm_s = sc;
  c->gm_partial = part;
  c->gm_h = hh;
  c->gm_cap = cap;
  return DGMG_OK;
}

}  // namespace

DGMG_API dgmg_status dgmg_gmres_solve(dgmg_ctx* c, const double* b, double* x, double rtol, int maxit,
                                      int* iters, double* hist) {
  RET(check_level(c, c ? c->L : 0, 0, 1));
  if (!x || !b || !iters || !hist) return fail(c, DGMG_ERR_ARG, "null argument");
  if (!(rtol > 0) || maxit < 1 || maxit > 1000)
    return fail(c, DGMG_ERR_ARG, "rtol must be > 0 and 1 <= maxit <= 1000");
  RET(ensure_gmres(c, maxit < 16 ? maxit : 16, 0, 0));
  const long long n = c->lv[c->L].ndof;
  hipStream_t s = c->stream;
  // device scalars: cap + 1 first-pass coefficients h1, cap + 1 second-pass
  // coefficients h2, |w|^2 (and |b|^2 at the start) nn; pinned mirror hh
  int cap = 0;
  double *h1 = nullptr, *h2 = nullptr, *nn = nullptr, *hh = nullptr;
  auto bind = [&]() {
    cap = c->gm_cap;
    h1 = c->gm_s;
    h2 = c->gm_s + (cap + 2);
    nn = c->gm_s + 2 * (cap + 2);
    hh = c->gm_h;
  };
  bind();
  // |b|, V_0 = b / |b|
  HIPCHK(c, dgmg::blas_dot2(b, b, nullptr, nullptr, n, 1, c->gm_partial, nullptr, nn, nullptr, s));
  HIPCHK(c, hipMemcpyAsync(hh, nn, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  const double beta = std::sqrt(hh[0]);
  if (!std::isfinite(beta)) return fail(c, DGMG_ERR_ARG, "right-hand side contains NaN/Inf");
  *iters = 0;
  hist[0] = 1.0;
  RET(zero_vec<double>(c, x, n));
  if (beta == 0) return DGMG_OK;
  HIPCHK(c, dgmg::blas_normalise(c->gm_V, c->r, b, nn, n, s));
  // Hessenberg matrix (column-major, (maxit + 1) x maxit), Givens rotations,
  // and the rotated right-hand side g
  std::vector<double> H((size_t)(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), g(maxit + 1, 0.0);
  g[0] = beta;
  int m = 0;
  dgmg_status status = DGMG_ERR_NOT_CONVERGED;
  for (int j = 0; j < maxit; ++j) {
    if (j + 1 > c->gm_cap) {  // grow: keep v_0..v_j and z_0..z_{j-1}
      int want = 2 * c->gm_cap < maxit ? 2 * c->gm_cap : maxit;
      size_t freeb = 0, totalb = 0;
      HIPCHK(c, hipMemGetInfo(&freeb, &totalb));
      // the new basis is allocated while the old one is still held
      const double fit = (0.9 * (double)freeb / (8.0 * (double)n) - 1.0) / 2.0;
      if (fit < want) want = (int)fit;
      if (want <= c->gm_cap)
        return fail(c, DGMG_ERR_ALLOC, "GMRES basis does not fit in device memory");
      RET(ensure_gmres(c, want, j + 1, j));
      bind();
    }
    double* zj = c->gm_Z + (long long)j * n;
    // z_j = V(v_j) through the CG workspace (graph replay), w = A z_j in q.
    // The captured V-cycle reads r and writes z: v_j was written into r as
    // well when it was normalised, z_j is copied out of z (cheaper than
    // running the ~80 launches of a V-cycle on z_j directly: on a stream a
    // launch costs ~0.7 us more than in a graph; a 3-D Q3 32^3 vector copies
    // in ~7 us).
    RET(precondition_cg(c, 1));
    HIPCHK(c, hipMemcpyAsync(zj, c->z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    RET(op_apply<double>(c, c->L, zj, c->q, 1));
    // classical Gram-Schmidt, twice: h = V^T w, w -= V h
    HIPCHK(c, dgmg::blas_multi_dot(c->gm_V, c->q, n, j + 1, c->gm_partial, h1, s));
    HIPCHK(c, dgmg::blas_multi_axpy(c->q, c->gm_V, h1, j + 1, -1.0, n, s));
    HIPCHK(c, dgmg::blas_multi_dot(c->gm_V, c->q, n, j + 1, c->gm_partial, h2, s));
    HIPCHK(c, dgmg::blas_multi_axpy(c->q, c->gm_V, h2, j + 1, -1.0, n, s));
    HIPCHK(c, dgmg::blas_dot2(c->q, c->q, nullptr, nullptr, n, 1, c->gm_partial, nullptr, nn,
                              nullptr, s));
    HIPCHK(c, hipMemcpyAsync(hh, c->gm_s, sizeof(double) * 3 * (cap + 2), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipEventRecord(c->ev_check, s));
    RET(poll_event(c, c->ev_check));
    double* Hj = &H[(size_t)j * (maxit + 1)];
    for (int i = 0; i <= j; ++i) Hj[i] = hh[i] + hh[cap + 2 + i];
    const double w2 = hh[2 * (cap + 2)];
    if (!std::isfinite(w2) || !(w2 >= 0)) return fail(c, DGMG_ERR_BREAKDOWN, "GMRES: non-finite Arnoldi scalar");
    Hj[j + 1] = std::sqrt(w2);
    if (w2 > 0 && j + 1 < maxit)
      HIPCHK(c, dgmg::blas_normalise(c->gm_V + (long long)(j + 1) * n, c->r, c->q, nn, n, s));
    // apply the previous rotations to the new column, then a new one
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
      Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
      Hj[i] = t;
    }
    const double den = std::hypot(Hj[j], Hj[j + 1]);
    if (!(den > 0)) return fail(c, DGMG_ERR_BREAKDOWN, "GMRES: singular Hessenberg column");
    cs[j] = Hj[j] / den;
    sn[j] = Hj[j + 1] / den;
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    m = j + 1;
    hist[m] = std::fabs(g[m]) / beta;
    *iters = m;
    if (hist[m] <= rtol || w2 == 0) {
      status = DGMG_OK;
      break;
    }
  }
  // y = R^{-1} g (back substitution), x = Z y
  std::vector<double> y(m);
  for (int i = m - 1; i >= 0; --i) {
    double sum = g[i];
    for (int l = i + 1; l < m; ++l) sum -= H[(size_t)l * (maxit + 1) + i] * y[l];
    y[i] = sum / H[(size_t)i * (maxit + 1) + i];
  }
  for (int i = 0; i < m; ++i) hh[i] = y[i];
  HIPCHK(c, hipMemcpyAsync(h1, hh, sizeof(double) * m, hipMemcpyHostToDevice, s));
  HIPCHK(c, dgmg::blas_multi_axpy(x, c->gm_Z, h1, m, 1.0, n, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (status != DGMG_OK) c->err = "maximum number of iterations reached";
  return status;
}

DGMG_API dgmg_status dgmg_dot(dgmg_ctx* c, int level, const double* a, const double* b, int nrhs,
                              double* out) {
  RET(check_level(c, level, 0, nrhs));
  if (!a || !b || !out) return fail(c, DGMG_ERR_ARG, "null argument");
  double* res = c->scal + S_ZQ * c->nrhs_max;
  HIPCHK(c, dgmg::blas_dot2(a, b, nullptr, nullptr, c->lv[level].ndof, nrhs, c->partial, nullptr,
                            res, nullptr, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->hbuf, res, sizeof(double) * nrhs, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipEventRecord(c->ev_check, c->stream));
  RET(poll_event(c, c->ev_check));
  std::memcpy(out, c->hbuf, sizeof(double) * nrhs);
  return DGMG_OK;
}

DGMG_API dgmg_status dgmg_adjoint_dkappa(dgmg_ctx* c, const double* lam, const double* u, int nrhs,
                                         double* per_rhs, double* total) {
  RET(check_level(c, c ? c->L : 0, 0, nrhs));
  if (!lam || !u || !total) return fail(c, DGMG_ERR_ARG, "null argument");
  const long long n = c->lv[c->L].ndof;
  // A_1 u in the CG workspace q, first-stage partial sums of lambda . A_1 u,
  // then the negated sums and their total on the device
  RET(op_apply_unit(c, c->L, u, c->q, nrhs));
  HIPCHK(c, dgmg::blas_dot2(lam, c->q, nullptr, nullptr, n, nrhs, c->partial, nullptr, nullptr, nullptr,
                            c->stream));
  HIPCHK(c, dgmg::blas_neg_finalize_sum(c->partial, n, nrhs, c->dk, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->hbuf, c->dk, sizeof(double) * (nrhs + 1), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipEventRecord(c->ev_check, c->stream));
  RET(poll_event(c, c->ev_check));
  if (per_rhs) std::memcpy(per_rhs, c->hbuf, sizeof(double) * nrhs);
  *total = c->hbuf[nrhs];
  return DGMG_OK;
}

namespace {

// ---------------------------------------------------------------- autotuner
// Times every workgroup shape x XCD numbering of apply and smooth on the
// finest level with HIP events (best of three batches) and keeps the fastest.
// Results are cached in a JSON object, one entry per line:
//   "gfx950/d3/k3/L4/nrhs16/fp64/smooth": {"shape": 0, "remap": 1, "us": 16.50},

std::string tune_key(const dgmg_ctx* c, int nrhs, int prec, const char* kernel) {
  char buf[128];
  std::snprintf(buf, sizeof(buf), "gfx950/d%d/k%d/L%d/nrhs%d/fp%d/%s", c->dim, c->k, c->L, nrhs, prec,
                kernel);
  return buf;
}

struct CacheEntry {
  std::string key;
  int shape, remap;
  double us;
};

std::vector<CacheEntry> read_cache(const char* path) {
  std::vector<CacheEntry> out;
  if (!path) return out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    char key[256];
    CacheEntry e;
    if (std::sscanf(line, " \"%255[^\"]\": {\"shape\": %d, \"remap\": %d, \"us\": %lf", key, &e.shape,
                    &e.remap, &e.us) == 4) {
      e.key = key;
      out.push_back(e);
    }
  }
  std::fclose(f);
  return out;
}

void write_cache(const char* path, const std::vector<CacheEntry>& es) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < es.size(); ++i)
    std::fprintf(f, "  \"%s\": {\"shape\": %d, \"remap\": %d, \"us\": %.3f}%s\n", es[i].key.c_str(),
                 es[i].shape, es[i].remap, es[i].us, i + 1 < es.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

template <typename T>
dgmg_status tune_kernel(dgmg_ctx* c, int nrhs, bool smooth, int level, T* x, T* y,
                        dgmg_ctx::Tuning& slot) {
  // candidate shapes; those that would repeat another are left out
  std::vector<int> shapes;
  const KernelSet<T>& ks = kset<T>(c);
  const bool rpack = nrhs > 1 && (smooth ? ks.smooth_rpack : ks.apply_rpack);
  if (smooth) {
    const bool hi = c->variant == DGMG_SMOOTH_FULL ? ks.smooth_hi_full : ks.smooth_split;
    for (int v = 0; v < (hi ? 8 : 4); ++v) shapes.push_back(v);
    if (rpack)
      for (int v = 8; v < 12; ++v) shapes.push_back(v);
  } else {
    shapes = {0, 1};
    if (ks.apply_rf) shapes.push_back(2);
    if (rpack) shapes.push_back(3);
  }
  const int reps = smooth ? 3 : 20;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  double best = 1e300;
  dgmg_ctx::Tuning pick = slot;
  for (int shape : shapes)
    for (int remap = 0; remap < 2; ++remap) {
      slot.shape = shape;
      slot.remap = remap;
      double t_best = 1e300;
      for (int trial = 0; trial < 4; ++trial) {  // trial 0 warms up
        HIPCHK(c, hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r) {
          if (smooth) RET(op_smooth<T>(c, level, x, y, 0, nrhs));
          else RET(op_apply<T>(c, level, x, y, nrhs));
        }
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        const double us = 1e3 * ms / reps;
        if (trial > 0 && us < t_best) t_best = us;
      }
      if (t_best < best) {
        best = t_best;
        pick.shape = shape;
        pick.remap = remap;
        pick.us = t_best;
      }
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  slot = pick;
  return DGMG_OK;
}

}  // namespace

DGMG_API dgmg_status dgmg_autotune(dgmg_ctx* c, int nrhs, const char* cache_path, char* report,
                                   int report_len) {
  RET(check_level(c, c ? c->L : 0, 0, nrhs));
  std::vector<CacheEntry> cache = read_cache(cache_path);
  std::string rep;
  bool dirty = false;
  // decisions: the CG's FP64 apply on the finest level, and the smoother of
  // the V-cycle's precision on every level it runs on
  struct Job {
    int prec;
    bool smooth;
    int level;
  };
  std::vector<Job> jobs{{64, false, c->L}};
  for (int l = 1; l <= c->L; ++l) jobs.push_back({c->prec, true, l});
  if (c->prec == 64) RET(ensure_levels<double>(c, c->L - 1));
  else RET(ensure_levels<float>(c, c->L));
  for (const Job& jb : jobs) {
    char kname[32];
    if (jb.smooth) std::snprintf(kname, sizeof(kname), "smooth/l%d", jb.level);
    else std::snprintf(kname, sizeof(kname), "apply");
    const std::string key = tune_key(c, nrhs, jb.prec, kname);
    const int pi = jb.prec == 64 ? 0 : 1;
    dgmg_ctx::Tuning& slot = jb.smooth ? c->tune_smooth[pi][jb.level] : c->tune_apply[pi];
    const int nshapes = jb.smooth ? dgmg::kSmoothShapes : dgmg::kApplyShapes;
    bool found = false;
    for (const CacheEntry& e : cache)
      if (e.key == key && e.shape >= 0 && e.shape < nshapes && (e.remap == 0 || e.remap == 1)) {
        slot.shape = e.shape;
        slot.remap = e.remap;
        slot.us = e.us;
        found = true;
      }
    if (!found) {
      Level& Lv = c->lv[jb.level];
      const long long n = Lv.ndof * nrhs;
      if (jb.prec == 64) {
        double* x = jb.level == c->L ? c->p : Lv.x64;
        double* y = jb.level == c->L ? (jb.smooth ? c->r : c->q) : Lv.b64;
        RET(zero_vec<double>(c, x, n));
        RET(zero_vec<double>(c, y, n));
        RET(tune_kernel<double>(c, nrhs, jb.smooth, jb.level, x, y, slot));
      } else {
        RET(zero_vec<float>(c, Lv.x32, n));
        RET(zero_vec<float>(c, Lv.b32, n));
        RET(tune_kernel<float>(c, nrhs, jb.smooth, jb.level, Lv.x32, Lv.b32, slot));
      }
      cache.push_back({key, slot.shape, slot.remap, slot.us});
      dirty = true;
    }
    char line[256];
    std::snprintf(line, sizeof(line), "%s shape=%d remap=%d us=%.3f%s\n", key.c_str(), slot.shape,
                  slot.remap, slot.us, found ? " (cached)" : "");
    rep += line;
  }
  if (dirty) write_cache(cache_path, cache);
  drop_graphs(c);  // graphs hold the previous launch shapes
  if (report && report_len > 0) {
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return DGMG_OK;
}

DGMG_API dgmg_status dgmg_patch_eigen(int degree, double sigma, int smoother_variant, int type,
                                      double* S, double* lam) {
  if (degree < 1 || degree > dgmg::kMaxDegree || !(sigma > 0) || type < 0 || type > 3 || !S || !lam)
    return DGMG_ERR_ARG;
  if (smoother_variant != DGMG_SMOOTH_EXACT && smoother_variant != DGMG_SMOOTH_LOCAL &&
      smoother_variant != DGMG_SMOOTH_FULL && smoother_variant != DGMG_SMOOTH_CLAMPED)
    return DGMG_ERR_ARG;
  if (smoother_variant == DGMG_SMOOTH_CLAMPED && degree < 3) return DGMG_ERR_ARG;
  dgmg::HostTables H;
  const char* err = nullptr;
  if (!dgmg::build_host_tables(degree, sigma, H, &err)) return DGMG_ERR_ARG;
  const std::vector<double>* Ss = H.S;
  const std::vector<double>* Ls = H.lam;
  if (smoother_variant == DGMG_SMOOTH_FULL) { Ss = H.Sf; Ls = H.lamf; }
  if (smoother_variant == DGMG_SMOOTH_CLAMPED) { Ss = H.Sc; Ls = H.lamc; }
  std::memcpy(S, Ss[type].data(), sizeof(double) * H.E * H.E);
  std::memcpy(lam, Ls[type].data(), sizeof(double) * H.E);
  return DGMG_OK;
}

DGMG_API const char* dgmg_last_error(const dgmg_ctx* c) {
  return c ? c->err.c_str() : "null context";
}

DGMG_API dgmg_status dgmg_destroy(dgmg_ctx* c) {
  if (!c) return DGMG_ERR_ARG;
  if (c->ready) hipStreamSynchronize(c->stream);
  drop_graphs(c);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  for (Level& L : c->lv) {
    hipFree(L.b64);
    hipFree(L.x64);
    hipFree(L.b32);
    hipFree(L.x32);
    hipFree(L.alt64);
    hipFree(L.alt32);
  }
  hipFree(c->tab64);
  hipFree(c->tab32);
  hipFree(c->dense64);
  hipFree(c->dense32);
  hipFree(c->dense_part);
  hipFree(c->r);
  hipFree(c->z);
  hipFree(c->p);
  hipFree(c->q);
  hipFree(c->scal);
  hipFree(c->partial);
  hipFree(c->partial2);
  hipFree(c->active);
  hipFree(c->nb);
  hipFree(c->dk);
  free_gmres(c);
  if (c->hbuf) hipHostFree(c->hbuf);
  if (c->hact) hipHostFree(c->hact);
  if (c->hnb) hipHostFree(c->hnb);
  if (c->rec) hipHostFree(c->rec);
  if (c->ev_check) hipEventDestroy(c->ev_check);
  delete c;
  return DGMG_OK;
}
