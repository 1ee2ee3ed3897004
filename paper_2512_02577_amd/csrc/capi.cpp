// C interface of libpmg (declared in include/pmg.h): host setup, device buffers, and the
// orchestration of the h-multigrid V-cycle and the flexible CG on one HIP stream.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>
#include <vector>

#include "dispatch.h"
#include "host_tables.h"
#include "launch.h"
#include "pmg.h"

using namespace pmg;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define PMG_TRY(expr)                                                        \
  do {                                                                       \
    int rc_ = (expr);                                                        \
    if (rc_ != 0) return fail(rc_ == -3 ? PMG_ERR_OUT_OF_MEMORY : PMG_ERR_DEVICE, "%s failed (%d): %s", #expr, rc_, \
                              hipGetErrorString(hipGetLastError()));         \
  } while (0)

#define PMG_HIP(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(e_ == hipErrorOutOfMemory ? PMG_ERR_OUT_OF_MEMORY : PMG_ERR_DEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                                     \
  } while (0)

template <typename T>
struct PrecData {
  DevTabs<T> tabs{};
  std::vector<T *> r, z, t;   // per h-level work vectors
  T *tw1 = nullptr, *tw2 = nullptr;  // intermediates of the 1D transfer passes
};

}  // namespace

struct pmg_mesh {
  int dim = 3, n = 0;
  std::vector<int> sizes;  // cells per direction, coarsest first
};

struct pmg_problem {
  int dim = 3, p = 1, hcode = 0;
  std::vector<int> sizes, degrees;
  pmg_config cfg{};
  Tables tab;
  // device state
  bool dev = false;
  int device = -1;
  std::vector<void *> allocs;
  PrecData<double> d64;
  PrecData<float> d32;
  double *S0 = nullptr, *lam0 = nullptr, *cw1 = nullptr, *cw2 = nullptr;
  double *fr[2] = {nullptr, nullptr}, *fz = nullptr, *fp = nullptr, *fq = nullptr;
  double *part = nullptr, *scal = nullptr, *hscal = nullptr;
  Arena arena;

  long nodes(int l) const {
    long m = (long)p * sizes[l] + 1;
    return dim == 3 ? m * m * m : m * m;
  }
  int finest() const { return (int)sizes.size() - 1; }
  double cscale(int l) const { return dim == 3 ? 1.0 / sizes[l] : 1.0; }
  template <typename T>
  PrecData<T> &pd();
};

template <>
PrecData<double> &pmg_problem::pd<double>() { return d64; }
template <>
PrecData<float> &pmg_problem::pd<float>() { return d32; }

namespace {

int check_ready(const pmg_problem *pr) {
  if (!pr) return fail(PMG_ERR_INVALID_ARG, "problem is NULL");
  if (!pr->dev) return fail(PMG_ERR_STATE, "pmg_device_init has not been called");
  return PMG_OK;
}

int check_level(const pmg_problem *pr, int hlevel) {
  if (hlevel < 0 || hlevel >= (int)pr->sizes.size())
    return fail(PMG_ERR_INVALID_ARG, "hlevel %d out of range [0, %d)", hlevel, (int)pr->sizes.size());
  return PMG_OK;
}

int check_prec(int prec) {
  if (prec != PMG_FP64 && prec != PMG_FP32) return fail(PMG_ERR_INVALID_ARG, "precision %d unknown", prec);
  return PMG_OK;
}

template <typename T>
int do_apply(pmg_problem *pr, int l, bool resid, const T *b, const T *u, T *out, hipStream_t s) {
  const int tc = tile_cells(pr->p);
  ApplyArgs<T> a{};
  a.Kt = pr->pd<T>().tabs.Kt;
  a.Mt = pr->pd<T>().tabs.Mt;
  a.c = (T)pr->cscale(l);
  a.n = pr->sizes[l];
  a.ntile = (a.n + tc - 1) / tc;
  a.n_tiles = pr->dim == 3 ? a.ntile * a.ntile * a.ntile : a.ntile * a.ntile;
  a.u = u;
  a.b = b;
  a.out = out;
  PMG_TRY(launch_apply<T>(pr->dim, pr->p, resid, a, pr->arena, s));
  return PMG_OK;
}

template <typename T>
SmoothArgs<T> smooth_args(pmg_problem *pr, int l) {
  SmoothArgs<T> a{};
  a.tb = pr->pd<T>().tabs;
  a.c = (T)pr->cscale(l);
  a.cinv = (T)(1.0 / pr->cscale(l));
  a.n = pr->sizes[l];
  a.full = pr->cfg.local_solver == PMG_LOCAL_FULL_V;
  a.n_iter = pr->cfg.n_local_iter;
  return a;
}

template <typename T>
int do_smooth(pmg_problem *pr, int l, int dir, T *u, const T *b, hipStream_t s) {
  SmoothArgs<T> base = smooth_args<T>(pr, l);
  base.u = u;
  base.b = b;
  const int n = pr->sizes[l], ncol = 1 << pr->dim;
  for (int ci = 0; ci < ncol; ++ci) {
    const int col = dir > 0 ? ci : ncol - 1 - ci;
    SmoothArgs<T> a = base;
    a.n_patch = 1;
    for (int d = 0; d < 3; ++d) {
      if (d >= pr->dim) {
        a.first[d] = 0;
        a.cnt[d] = 1;
        continue;
      }
      const int bit = (col >> d) & 1;
      a.first[d] = bit ? 1 : 2;
      a.cnt[d] = a.first[d] <= n - 1 ? (n - 1 - a.first[d]) / 2 + 1 : 0;
      a.n_patch *= a.cnt[d];
    }
    if (a.n_patch == 0) continue;
    PMG_TRY(launch_smooth_color<T>(pr->dim, pr->p, pr->hcode, a, pr->arena, s));
  }
  return PMG_OK;
}

template <typename T>
int do_restrict(pmg_problem *pr, int l, const T *fine, T *coarse, hipStream_t s) {
  TransferArgs<T> a{};
  a.W1 = pr->pd<T>().tabs.W1;
  a.Wr = pr->pd<T>().tabs.Wr;
  a.nc = pr->sizes[l - 1];
  a.in = fine;
  a.out = coarse;
  a.w1 = pr->pd<T>().tw1;
  a.w2 = pr->pd<T>().tw2;
  PMG_TRY(launch_restrict<T>(pr->dim, pr->p, a, s));
  return PMG_OK;
}

template <typename T>
int do_prolong(pmg_problem *pr, int l, const T *coarse, T *fine, hipStream_t s) {
  TransferArgs<T> a{};
  a.W1 = pr->pd<T>().tabs.W1;
  a.Wr = pr->pd<T>().tabs.Wr;
  a.nc = pr->sizes[l - 1];
  a.in = coarse;
  a.out = fine;
  a.w1 = pr->pd<T>().tw1;
  a.w2 = pr->pd<T>().tw2;
  PMG_TRY(launch_prolong_add<T>(pr->dim, pr->p, a, s));
  return PMG_OK;
}

template <typename T>
int do_coarse(pmg_problem *pr, const T *r, T *z, hipStream_t s) {
  CoarseArgs<T> a{};
  a.S = pr->S0;
  a.lam = pr->lam0;
  a.c0inv = 1.0 / pr->cscale(0);
  a.m = pr->tab.m0;
  a.mt = pr->tab.m0 + 2;
  a.r = r;
  a.z = z;
  a.w1 = pr->cw1;
  a.w2 = pr->cw2;
  PMG_TRY(launch_coarse<T>(pr->dim, a, s));
  return PMG_OK;
}

// h-multigrid V(n_pre, n_post) from a zero guess on the finest level (Sec. 2).
template <typename T>
int do_vcycle(pmg_problem *pr, const T *r, T *z, hipStream_t s) {
  const int L = pr->finest();
  PrecData<T> &w = pr->pd<T>();
  if (L == 0) return do_coarse<T>(pr, r, z, s);
  for (int l = L; l >= 1; --l) {
    const T *R = l == L ? r : w.r[l];
    T *Z = l == L ? z : w.z[l];
    const int m = pr->p * pr->sizes[l] + 1;
    PMG_TRY(launch_init_z<T>(pr->dim, m, Z, R, s));
    for (int k = 0; k < pr->cfg.n_pre; ++k) {
      int rc = do_smooth<T>(pr, l, +1, Z, R, s);
      if (rc) return rc;
    }
    int rc = do_apply<T>(pr, l, true, R, Z, w.t[l], s);
    if (rc) return rc;
    rc = do_restrict<T>(pr, l, w.t[l], w.r[l - 1], s);
    if (rc) return rc;
  }
  int rc = do_coarse<T>(pr, w.r[0], w.z[0], s);
  if (rc) return rc;
  for (int l = 1; l <= L; ++l) {
    const T *R = l == L ? r : w.r[l];
    T *Z = l == L ? z : w.z[l];
    rc = do_prolong<T>(pr, l, w.z[l - 1], Z, s);
    if (rc) return rc;
    for (int k = 0; k < pr->cfg.n_post; ++k) {
      rc = do_smooth<T>(pr, l, -1, Z, R, s);
      if (rc) return rc;
    }
  }
  return PMG_OK;
}

int vcycle_any(pmg_problem *pr, int mg_prec, const double *r, double *z, hipStream_t s) {
  if (mg_prec == PMG_FP64) return do_vcycle<double>(pr, r, z, s);
  const int L = pr->finest();
  const long N = pr->nodes(L);
  PMG_TRY(launch_cast_d2f(r, pr->d32.r[L], N, s));
  int rc = do_vcycle<float>(pr, pr->d32.r[L], pr->d32.z[L], s);
  if (rc) return rc;
  PMG_TRY(launch_cast_f2d(pr->d32.z[L], z, N, s));
  return PMG_OK;
}

template <typename T>
void bind_tabs(DevTabs<T> &d, const Tables &t, T *base, const std::vector<size_t> &off) {
  size_t k = 0;
  for (size_t l = 0; l < t.lev.size(); ++l) {
    d.Kp[l] = base + off[k++];
    d.Mp[l] = base + off[k++];
    d.invD[l] = base + off[k++];
    d.Tp[l] = base + off[k++];
    d.TpT[l] = base + off[k++];
  }
  d.Kr = base + off[k++];
  d.Mr = base + off[k++];
  d.Kt = base + off[k++];
  d.Mt = base + off[k++];
  d.W1 = base + off[k++];
  d.Wr = base + off[k++];
}

// concatenated tables (each block padded to 32 entries) and their offsets
void flatten_tabs(const Tables &t, std::vector<double> &flat, std::vector<size_t> &off) {
  auto put = [&](const dvec &v) {
    off.push_back(flat.size());
    flat.insert(flat.end(), v.begin(), v.end());
    flat.resize((flat.size() + 31) / 32 * 32 + 32, 0.0);
  };
  for (const PLevel &L : t.lev) {
    put(L.Kp);
    put(L.Mp);
    put(L.invD);
    put(L.Tp);
    put(L.TpT);
  }
  put(t.Kr);
  put(t.Mr);
  put(t.Kt);
  put(t.Mt);
  put(t.W1);
  put(t.Wr);
}

template <typename T>
int dev_alloc(pmg_problem *pr, T **out, size_t count) {
  void *ptr = nullptr;
  PMG_HIP(hipMalloc(&ptr, count * sizeof(T) + 64));
  pr->allocs.push_back(ptr);
  *out = reinterpret_cast<T *>(ptr);
  return PMG_OK;
}

void release(pmg_problem *pr) {
  for (void *ptr : pr->allocs) (void)hipFree(ptr);
  pr->allocs.clear();
  if (pr->hscal) (void)hipHostFree(pr->hscal);
  pr->hscal = nullptr;
  pr->dev = false;
}

}  // namespace

extern "C" {

const char *pmg_last_error(void) { return g_err.c_str(); }

void pmg_default_config(pmg_config *cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->local_solver = PMG_LOCAL_HALF_V;
  cfg->n_local_iter = 1;
  cfg->n_pre = 1;
  cfg->n_post = 1;
  cfg->max_iter = 200;
  cfg->rtol = 1e-8;
  cfg->n_omega = 0;
}

int pmg_setup_mesh(int dim, int n, int n_hlevels, const double *vertices, pmg_mesh **out) {
  if (!out) return fail(PMG_ERR_INVALID_ARG, "out is NULL");
  if (dim != 2 && dim != 3) return fail(PMG_ERR_INVALID_ARG, "dim must be 2 or 3, got %d", dim);
  if (n < 2 || n > 1024) return fail(PMG_ERR_INVALID_ARG, "n must be in [2, 1024], got %d", n);
  if (n_hlevels < 0) return fail(PMG_ERR_INVALID_ARG, "n_hlevels must be >= 0");
  if (vertices) return fail(PMG_ERR_UNSUPPORTED, "distorted meshes are not supported by this build");
  std::vector<int> sizes{n};
  while (sizes.back() % 2 == 0 && sizes.back() > 3 && (n_hlevels == 0 || (int)sizes.size() < n_hlevels))
    sizes.push_back(sizes.back() / 2);
  if (n_hlevels && (int)sizes.size() != n_hlevels)
    return fail(PMG_ERR_INVALID_ARG, "cannot build %d nested levels from n = %d", n_hlevels, n);
  try {
    pmg_mesh *m = new pmg_mesh;
    m->dim = dim;
    m->n = n;
    m->sizes.assign(sizes.rbegin(), sizes.rend());
    *out = m;
  } catch (const std::exception &e) {
    return fail(PMG_ERR_OUT_OF_MEMORY, "%s", e.what());
  }
  return PMG_OK;
}

int pmg_mesh_levels(const pmg_mesh *m, int *dim, int *n_hlevels, int32_t *n_cells) {
  if (!m) return fail(PMG_ERR_INVALID_ARG, "mesh is NULL");
  if (dim) *dim = m->dim;
  if (n_hlevels) *n_hlevels = (int)m->sizes.size();
  if (n_cells)
    for (size_t i = 0; i < m->sizes.size(); ++i) n_cells[i] = m->sizes[i];
  return PMG_OK;
}

void pmg_destroy_mesh(pmg_mesh *m) { delete m; }

int pmg_setup_dofmap(const pmg_mesh *m, int degree, const int32_t *p_levels, int n_plevels, const pmg_config *cfg,
                     pmg_problem **out) {
  if (!m || !out) return fail(PMG_ERR_INVALID_ARG, "mesh or out is NULL");
  if (degree < 1 || degree > kMaxDegree) return fail(PMG_ERR_INVALID_ARG, "degree must be in [1, 8], got %d", degree);
  std::vector<int> deg;
  if (p_levels) {
    if (n_plevels < 1 || n_plevels > 4) return fail(PMG_ERR_INVALID_ARG, "n_plevels must be in [1, 4]");
    for (int i = 0; i < n_plevels; ++i) deg.push_back(p_levels[i]);
    for (int i = 1; i < n_plevels; ++i)
      if (deg[i] <= deg[i - 1]) return fail(PMG_ERR_INVALID_ARG, "p_levels must be strictly ascending");
    if (deg.front() != 1 || deg.back() != degree)
      return fail(PMG_ERR_INVALID_ARG, "p_levels must start at 1 and end at the degree");
  } else {
    for (int x = 1; x < degree; x = 2 * x + 1) deg.push_back(x);
    deg.push_back(degree);
  }
  const int hcode = hierarchy_code(degree, deg.data(), (int)deg.size());
  if (hcode < 0) return fail(PMG_ERR_UNSUPPORTED, "this p-level list is not compiled in");
  pmg_config c;
  pmg_default_config(&c);
  if (cfg) c = *cfg;
  if (c.local_solver != PMG_LOCAL_HALF_V && c.local_solver != PMG_LOCAL_FULL_V)
    return fail(PMG_ERR_INVALID_ARG, "local_solver unknown");
  if (c.n_local_iter < 1 || c.n_local_iter > 64) return fail(PMG_ERR_INVALID_ARG, "n_local_iter must be in [1, 64]");
  if (c.n_pre < 0 || c.n_post < 0 || c.n_pre > 16 || c.n_post > 16)
    return fail(PMG_ERR_INVALID_ARG, "n_pre and n_post must be in [0, 16]");
  if (c.max_iter < 1) return fail(PMG_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (!(c.rtol > 0.0) || !(c.rtol < 1.0)) return fail(PMG_ERR_INVALID_ARG, "rtol must be in (0, 1)");
  if (c.n_omega < 0 || c.n_omega > (int)deg.size()) return fail(PMG_ERR_INVALID_ARG, "n_omega out of range");
  for (int i = 1; i < c.n_omega; ++i)
    if (!(c.omega[i] > 0.0 && c.omega[i] < 2.0)) return fail(PMG_ERR_INVALID_ARG, "omega[%d] must be in (0, 2)", i);
  const long mm = (long)degree * m->n + 1;
  const double N = m->dim == 3 ? (double)mm * mm * mm : (double)mm * mm;
  if (N >= 2147483647.0) return fail(PMG_ERR_UNSUPPORTED, "more than 2^31 nodes");
  try {
    pmg_problem *pr = new pmg_problem;
    pr->dim = m->dim;
    pr->p = degree;
    pr->hcode = hcode;
    pr->sizes = m->sizes;
    pr->degrees = deg;
    pr->cfg = c;
    dvec om;
    if (c.n_omega > 0) om.assign(c.omega, c.omega + c.n_omega);
    build_tables(pr->dim, degree, deg, om, pr->sizes[0], pr->tab);
    *out = pr;
  } catch (const std::exception &e) {
    return fail(PMG_ERR_INVALID_ARG, "setup failed: %s", e.what());
  }
  return PMG_OK;
}

int pmg_problem_sizes(const pmg_problem *pr, int *dim, int *n_hlevels, int *n_plevels, int32_t *n_cells,
                      int64_t *n_nodes, int64_t *n_patches, int32_t *degrees, double *omega) {
  if (!pr) return fail(PMG_ERR_INVALID_ARG, "problem is NULL");
  if (dim) *dim = pr->dim;
  if (n_hlevels) *n_hlevels = (int)pr->sizes.size();
  if (n_plevels) *n_plevels = (int)pr->degrees.size();
  for (size_t l = 0; l < pr->sizes.size(); ++l) {
    if (n_cells) n_cells[l] = pr->sizes[l];
    if (n_nodes) n_nodes[l] = pr->nodes((int)l);
    if (n_patches) {
      long k = pr->sizes[l] - 1;
      n_patches[l] = pr->dim == 3 ? k * k * k : k * k;
    }
  }
  for (size_t i = 0; i < pr->degrees.size(); ++i) {
    if (degrees) degrees[i] = pr->degrees[i];
    if (omega) omega[i] = pr->tab.omega[i];
  }
  return PMG_OK;
}

int pmg_export_maps(const pmg_problem *pr, int hlevel, int plevel, int32_t *cell_dofs, int32_t *patch_interior,
                    int32_t *patch_closure, uint8_t *patch_color) {
  if (!pr) return fail(PMG_ERR_INVALID_ARG, "problem is NULL");
  if (int rc = check_level(pr, hlevel)) return rc;
  if (plevel < 0 || plevel >= (int)pr->degrees.size()) return fail(PMG_ERR_INVALID_ARG, "plevel out of range");
  const int dim = pr->dim, n = pr->sizes[hlevel], q = pr->degrees[plevel];
  const long m = (long)q * n + 1;
  const int ez = dim == 3 ? 1 : 0;
  auto node = [&](long i, long j, long k) { return (int32_t)(i + m * (j + m * k)); };
  if (cell_dofs) {
    const long nc = dim == 3 ? (long)n * n * n : (long)n * n, nl = dim == 3 ? (long)(q + 1) * (q + 1) * (q + 1)
                                                                             : (long)(q + 1) * (q + 1);
    for (long c = 0; c < nc; ++c) {
      const long cx = c % n, cy = (c / n) % n, cz = ez ? c / ((long)n * n) : 0;
      for (long e = 0; e < nl; ++e) {
        const long a = e % (q + 1), b = (e / (q + 1)) % (q + 1), f = ez ? e / ((long)(q + 1) * (q + 1)) : 0;
        cell_dofs[c * nl + e] = node(q * cx + a, q * cy + b, q * cz + f);
      }
    }
  }
  const long k = n - 1, np = dim == 3 ? k * k * k : k * k;
  const long ni = 2 * q - 1, nc2 = 2 * q + 1;
  const long ndi = dim == 3 ? ni * ni * ni : ni * ni, ndc = dim == 3 ? nc2 * nc2 * nc2 : nc2 * nc2;
  for (long j = 0; j < np; ++j) {
    const long vx = j % k + 1, vy = (j / k) % k + 1, vz = ez ? j / (k * k) + 1 : 0;
    if (patch_color) patch_color[j] = (uint8_t)((vx % 2) + 2 * (vy % 2) + (ez ? 4 * (vz % 2) : 0));
    if (patch_interior)
      for (long e = 0; e < ndi; ++e) {
        const long a = e % ni, b = (e / ni) % ni, f = ez ? e / (ni * ni) : 0;
        patch_interior[j * ndi + e] = node(q * (vx - 1) + 1 + a, q * (vy - 1) + 1 + b, ez ? q * (vz - 1) + 1 + f : 0);
      }
    if (patch_closure)
      for (long e = 0; e < ndc; ++e) {
        const long a = e % nc2, b = (e / nc2) % nc2, f = ez ? e / (nc2 * nc2) : 0;
        patch_closure[j * ndc + e] = node(q * (vx - 1) + a, q * (vy - 1) + b, ez ? q * (vz - 1) + f : 0);
      }
  }
  return PMG_OK;
}

int pmg_device_init(pmg_problem *pr) {
  if (!pr) return fail(PMG_ERR_INVALID_ARG, "problem is NULL");
  if (pr->dev) return PMG_OK;
  PMG_HIP(hipGetDevice(&pr->device));
  int lds = 0, ncu = 0;
  PMG_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, pr->device));
  PMG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pr->device));
  pr->arena.lds_max = (size_t)lds;
  int rc = PMG_OK;
  auto bail = [&](int code) {
    release(pr);
    return code;
  };
  // tables in both precisions
  std::vector<double> flat;
  std::vector<size_t> off;
  flatten_tabs(pr->tab, flat, off);
  double *t64 = nullptr;
  float *t32 = nullptr;
  if ((rc = dev_alloc(pr, &t64, flat.size()))) return bail(rc);
  if ((rc = dev_alloc(pr, &t32, flat.size()))) return bail(rc);
  std::vector<float> flat32(flat.begin(), flat.end());
  if (hipMemcpy(t64, flat.data(), flat.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t32, flat32.data(), flat32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(PMG_ERR_DEVICE, "table upload failed"));
  bind_tabs(pr->d64.tabs, pr->tab, t64, off);
  bind_tabs(pr->d32.tabs, pr->tab, t32, off);
  // coarse fast diagonalization
  const int m0 = pr->tab.m0;
  const size_t m0d = pr->dim == 3 ? (size_t)m0 * m0 * m0 : (size_t)m0 * m0;
  if ((rc = dev_alloc(pr, &pr->S0, (size_t)m0 * m0)) || (rc = dev_alloc(pr, &pr->lam0, (size_t)m0)) ||
      (rc = dev_alloc(pr, &pr->cw1, m0d)) || (rc = dev_alloc(pr, &pr->cw2, m0d)))
    return bail(rc);
  if (hipMemcpy(pr->S0, pr->tab.S0.data(), pr->tab.S0.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pr->lam0, pr->tab.lam0.data(), pr->tab.lam0.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess)
    return bail(fail(PMG_ERR_DEVICE, "coarse table upload failed"));
  // per-level work vectors
  const int nh = (int)pr->sizes.size();
  pr->d64.r.assign(nh, nullptr);
  pr->d64.z.assign(nh, nullptr);
  pr->d64.t.assign(nh, nullptr);
  pr->d32.r.assign(nh, nullptr);
  pr->d32.z.assign(nh, nullptr);
  pr->d32.t.assign(nh, nullptr);
  for (int l = 0; l < nh; ++l) {
    const size_t N = (size_t)pr->nodes(l);
    if (l < nh - 1) {
      if ((rc = dev_alloc(pr, &pr->d64.r[l], N)) || (rc = dev_alloc(pr, &pr->d64.z[l], N))) return bail(rc);
    }
    if (l >= 1 && (rc = dev_alloc(pr, &pr->d64.t[l], N))) return bail(rc);
    if ((rc = dev_alloc(pr, &pr->d32.r[l], N)) || (rc = dev_alloc(pr, &pr->d32.z[l], N))) return bail(rc);
    if (l >= 1 && (rc = dev_alloc(pr, &pr->d32.t[l], N))) return bail(rc);
  }
  // transfer intermediates, sized by the finest pair of levels
  if (nh > 1) {
    const size_t mf = (size_t)pr->p * pr->sizes[nh - 1] + 1, mc = (size_t)pr->p * pr->sizes[nh - 2] + 1;
    const size_t w = pr->dim == 3 ? mf * mf * mc : mf * mc;
    if ((rc = dev_alloc(pr, &pr->d64.tw1, w)) || (rc = dev_alloc(pr, &pr->d64.tw2, w)) ||
        (rc = dev_alloc(pr, &pr->d32.tw1, w)) || (rc = dev_alloc(pr, &pr->d32.tw2, w)))
      return bail(rc);
  }
  // outer solver vectors
  const size_t NF = (size_t)pr->nodes(nh - 1);
  if ((rc = dev_alloc(pr, &pr->fr[0], NF)) || (rc = dev_alloc(pr, &pr->fr[1], NF)) ||
      (rc = dev_alloc(pr, &pr->fz, NF)) || (rc = dev_alloc(pr, &pr->fp, NF)) || (rc = dev_alloc(pr, &pr->fq, NF)) ||
      (rc = dev_alloc(pr, &pr->part, 2 * (size_t)kRedBlocks)) || (rc = dev_alloc(pr, &pr->scal, (size_t)S_COUNT)))
    return bail(rc);
  if (hipHostMalloc((void **)&pr->hscal, S_COUNT * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return bail(fail(PMG_ERR_OUT_OF_MEMORY, "pinned scalar buffer"));
  // global arena for kernels whose workgroup arena exceeds the LDS limit
  size_t need = 0;
  for (int prec = 0; prec < 2; ++prec) {
    size_t b1 = patch_arena_bytes(pr->dim, prec, pr->p, pr->hcode);
    size_t b2 = apply_arena_bytes(pr->dim, prec, pr->p);
    if (b1 > pr->arena.lds_max && b1 > need) need = b1;
    if (b2 > pr->arena.lds_max && b2 > need) need = b2;
  }
  if (need) {
    pr->arena.slots = 2 * (ncu > 0 ? ncu : 256);
    void *g = nullptr;
    if ((rc = dev_alloc(pr, (unsigned char **)&g, need * pr->arena.slots))) return bail(rc);
    pr->arena.global = g;
  }
  pr->dev = true;
  return PMG_OK;
}

int pmg_apply_operator(pmg_problem *pr, int hlevel, int prec, const void *u, void *v, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (!u || !v) return fail(PMG_ERR_INVALID_ARG, "u or v is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return do_apply<double>(pr, hlevel, false, nullptr, (const double *)u, (double *)v, s);
  return do_apply<float>(pr, hlevel, false, nullptr, (const float *)u, (float *)v, s);
}

int pmg_residual(pmg_problem *pr, int hlevel, int prec, const void *b, const void *u, void *r, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (!u || !b || !r) return fail(PMG_ERR_INVALID_ARG, "b, u or r is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return do_apply<double>(pr, hlevel, true, (const double *)b, (const double *)u, (double *)r, s);
  return do_apply<float>(pr, hlevel, true, (const float *)b, (const float *)u, (float *)r, s);
}

int pmg_smooth(pmg_problem *pr, int hlevel, int prec, int color_dir, void *u, const void *b, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (color_dir != 1 && color_dir != -1) return fail(PMG_ERR_INVALID_ARG, "color_dir must be +1 or -1");
  if (!u || !b) return fail(PMG_ERR_INVALID_ARG, "u or b is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return do_smooth<double>(pr, hlevel, color_dir, (double *)u, (const double *)b, s);
  return do_smooth<float>(pr, hlevel, color_dir, (float *)u, (const float *)b, s);
}

int pmg_local_solve(pmg_problem *pr, int hlevel, int prec, int first_patch, int n_patches, const void *r, void *d,
                    void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  const long k = pr->sizes[hlevel] - 1, np = pr->dim == 3 ? k * k * k : k * k;
  if (first_patch < 0 || n_patches < 0 || first_patch + (long)n_patches > np)
    return fail(PMG_ERR_INVALID_ARG, "patch range [%d, %d) outside [0, %ld)", first_patch, first_patch + n_patches, np);
  if (n_patches == 0) return PMG_OK;
  if (!r || !d) return fail(PMG_ERR_INVALID_ARG, "r or d is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) {
    SmoothArgs<double> a = smooth_args<double>(pr, hlevel);
    a.r_blocks = (const double *)r;
    a.d_blocks = (double *)d;
    a.first_patch = first_patch;
    PMG_TRY(launch_local_only<double>(pr->dim, pr->p, pr->hcode, a, n_patches, pr->arena, s));
  } else {
    SmoothArgs<float> a = smooth_args<float>(pr, hlevel);
    a.r_blocks = (const float *)r;
    a.d_blocks = (float *)d;
    a.first_patch = first_patch;
    PMG_TRY(launch_local_only<float>(pr->dim, pr->p, pr->hcode, a, n_patches, pr->arena, s));
  }
  return PMG_OK;
}

int pmg_restrict(pmg_problem *pr, int hlevel, int prec, const void *fine, void *coarse, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (hlevel < 1) return fail(PMG_ERR_INVALID_ARG, "restriction needs hlevel >= 1");
  if (!fine || !coarse) return fail(PMG_ERR_INVALID_ARG, "fine or coarse is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return do_restrict<double>(pr, hlevel, (const double *)fine, (double *)coarse, s);
  return do_restrict<float>(pr, hlevel, (const float *)fine, (float *)coarse, s);
}

int pmg_prolongate_add(pmg_problem *pr, int hlevel, int prec, const void *coarse, void *fine, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (hlevel < 1) return fail(PMG_ERR_INVALID_ARG, "prolongation needs hlevel >= 1");
  if (!fine || !coarse) return fail(PMG_ERR_INVALID_ARG, "fine or coarse is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return do_prolong<double>(pr, hlevel, (const double *)coarse, (double *)fine, s);
  return do_prolong<float>(pr, hlevel, (const float *)coarse, (float *)fine, s);
}

int pmg_coarse_solve(pmg_problem *pr, int prec, const void *r, void *z, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (!r || !z) return fail(PMG_ERR_INVALID_ARG, "r or z is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return do_coarse<double>(pr, (const double *)r, (double *)z, s);
  return do_coarse<float>(pr, (const float *)r, (float *)z, s);
}

int pmg_vcycle(pmg_problem *pr, int mg_prec, const double *r, double *z, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_prec(mg_prec)) return rc;
  if (!r || !z) return fail(PMG_ERR_INVALID_ARG, "r or z is NULL");
  return vcycle_any(pr, mg_prec, r, z, (hipStream_t)stream);
}

int pmg_solve(pmg_problem *pr, int mg_prec, const double *b, double *x, int x_is_initial_guess, pmg_solve_info *info,
              void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_prec(mg_prec)) return rc;
  if (!b || !x) return fail(PMG_ERR_INVALID_ARG, "b or x is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int L = pr->finest();
  const long N = pr->nodes(L);
  double *r = pr->fr[0], *rn = pr->fr[1], *z = pr->fz, *p = pr->fp, *q = pr->fq;
  double *part = pr->part, *scal = pr->scal, *h = pr->hscal;
  auto finish = [&](int status, int it, double rel) {
    if (info) {
      info->iterations = it;
      info->rel_residual = rel;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      info->status = status;
    }
    return status;
  };
  auto fetch = [&]() -> int {
    PMG_HIP(hipMemcpyAsync(h, scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
    PMG_HIP(hipStreamSynchronize(s));
    return PMG_OK;
  };
  PMG_TRY(launch_dot_partial(b, b, nullptr, N, part, s));
  PMG_TRY(launch_dot_final(part, 1, 0, S_BB, scal, s));
  if (x_is_initial_guess) {
    if (int rc = do_apply<double>(pr, L, true, b, x, r, s)) return rc;
  } else {
    PMG_HIP(hipMemsetAsync(x, 0, N * sizeof(double), s));
    PMG_TRY(launch_copy(r, b, N, s));
  }
  PMG_TRY(launch_dot_partial(r, r, nullptr, N, part, s));
  PMG_TRY(launch_dot_final(part, 1, 0, S_RR, scal, s));
  if (int rc = fetch()) return rc;
  const double nb = std::sqrt(h[S_BB]);
  if (nb == 0.0) {
    PMG_HIP(hipMemsetAsync(x, 0, N * sizeof(double), s));
    PMG_HIP(hipStreamSynchronize(s));
    return finish(PMG_OK, 0, 0.0);
  }
  double rel = std::sqrt(h[S_RR]) / nb;
  if (rel <= pr->cfg.rtol) return finish(PMG_OK, 0, rel);
  if (int rc = vcycle_any(pr, mg_prec, r, z, s)) return rc;
  PMG_TRY(launch_copy(p, z, N, s));
  PMG_TRY(launch_dot_partial(r, z, nullptr, N, part, s));
  PMG_TRY(launch_dot_final(part, 1, 0, S_RZ, scal, s));
  for (int it = 1; it <= pr->cfg.max_iter; ++it) {
    if (int rc = do_apply<double>(pr, L, false, nullptr, p, q, s)) return rc;
    PMG_TRY(launch_dot_partial(p, q, nullptr, N, part, s));
    PMG_TRY(launch_dot_final(part, 1, 1, 0, scal, s));
    PMG_TRY(launch_fcg_xr(x, r, rn, p, q, scal, N, part, s));
    PMG_TRY(launch_dot_final(part, 1, 0, S_RR, scal, s));
    if (int rc = fetch()) return rc;
    const double pq = h[S_PQ];
    rel = std::sqrt(h[S_RR]) / nb;
    if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rel)) {
      fail(PMG_ERR_BREAKDOWN, "flexible CG breakdown at iteration %d: (p, Ap) = %g", it, pq);
      return finish(PMG_ERR_BREAKDOWN, it, rel);
    }
    if (rel <= pr->cfg.rtol) return finish(PMG_OK, it, rel);
    if (it == pr->cfg.max_iter) break;
    if (int rc = vcycle_any(pr, mg_prec, rn, z, s)) return rc;
    PMG_TRY(launch_dot_partial(z, rn, r, N, part, s));
    PMG_TRY(launch_dot_final(part, 2, 2, 0, scal, s));
    PMG_TRY(launch_fcg_p(p, z, scal, N, s));
    std::swap(r, rn);
  }
  fail(PMG_ERR_NOT_CONVERGED, "no convergence in %d iterations (relative residual %g)", pr->cfg.max_iter, rel);
  return finish(PMG_ERR_NOT_CONVERGED, pr->cfg.max_iter, rel);
}

void pmg_destroy_problem(pmg_problem *pr) {
  if (!pr) return;
  release(pr);
  delete pr;
}

}  // extern "C"
