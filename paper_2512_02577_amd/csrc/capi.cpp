// C interface of libpmg (declared in include/pmg.h): host setup, device buffers, and the
// orchestration of the h-multigrid V-cycle and the flexible CG on one HIP stream.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include <hipsolver/hipsolver.h>

#include "dispatch.h"
#include "geometry.h"
#include "host_tables.h"
#include "launch.h"
#include "pmg.h"
#include "problem.h"
#include "tab_layout.h"

using namespace pmg;

namespace {

thread_local std::string g_err;

}  // namespace

// Work memory of pmg_vcycle_noalloc: one copy of this array on every GPU the library runs
// on, held until the process ends.  Host code never uses its name as an address (on the
// host it is only a stand-in for the symbol): the per-device address comes from
// hipGetSymbolAddress in resolve_scratch.
static __device__ __align__(256) unsigned char scratch[PMG_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Resolves the current device's address of `scratch` once per device (called by
// pmg_device_init, with the problem's device current).
int resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(PMG_ERR_UNSUPPORTED, "device index %d beyond the %d the library tracks", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return PMG_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(PMG_ERR_DEVICE, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
  g_scratch_ptr[device] = static_cast<char *>(ptr);
  return PMG_OK;
}

char *scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace

int pmg::fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

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

// Storage of the general path's stored operator data (metric, patch diagonals):
// the compute type, or bfloat16 (FP32 compute, 3D only).
enum Store { ST_NATIVE = 0, ST_BF16 = 1 };

int check_prec(int prec) {
  if (prec != PMG_FP64 && prec != PMG_FP32 && prec != PMG_FP32_BF16)
    return fail(PMG_ERR_INVALID_ARG, "precision %d unknown", prec);
  return PMG_OK;
}

int store_of(int prec) { return prec == PMG_FP32_BF16 ? ST_BF16 : ST_NATIVE; }

template <typename T>
const QTabDev<T> &qtab(pmg_problem *pr, int l);
template <>
const QTabDev<double> &qtab<double>(pmg_problem *pr, int l) { return pr->qt64[l]; }
template <>
const QTabDev<float> &qtab<float>(pmg_problem *pr, int l) { return pr->qt32[l]; }

template <typename S>
const S *metric_of(pmg_problem *pr, int hl, int pl);
template <>
const double *metric_of<double>(pmg_problem *pr, int hl, int pl) { return pr->G64[hl * pr->nplev() + pl]; }
template <>
const float *metric_of<float>(pmg_problem *pr, int hl, int pl) { return pr->G32[hl * pr->nplev() + pl]; }
template <>
const bf16 *metric_of<bf16>(pmg_problem *pr, int hl, int pl) { return pr->G16[hl * pr->nplev() + pl]; }

template <typename S>
const S *invd_of(pmg_problem *pr, int hl, int pl);
template <>
const double *invd_of<double>(pmg_problem *pr, int hl, int pl) { return pr->invD64[hl * pr->nplev() + pl]; }
template <>
const float *invd_of<float>(pmg_problem *pr, int hl, int pl) { return pr->invD32[hl * pr->nplev() + pl]; }
template <>
const bf16 *invd_of<bf16>(pmg_problem *pr, int hl, int pl) { return pr->invD16[hl * pr->nplev() + pl]; }

template <int DIM, typename T, typename S>
int metric_apply_dim(pmg_problem *pr, int hl, bool resid, const T *b, const T *u, T *out, hipStream_t s) {
  using ML = MetricLaunchers<DIM, T, S>;
  const int n = pr->sizes[hl], m = pr->p * n + 1, L = pr->nplev();
  PMG_TRY(ML::apply_init(m, resid, b, u, out, s));
  MetricApplyArgs<T, S> a{};
  a.qt = qtab<T>(pr, L - 1);
  a.G = metric_of<S>(pr, hl, L - 1);
  a.n = n;
  a.sign = resid ? T(-1) : T(1);
  a.u = u;
  a.out = out;
  for (int col = 0; col < (1 << DIM); ++col) {
    MetricApplyArgs<T, S> c = a;
    c.n_cells = 1;
    for (int d = 0; d < 3; ++d) {
      if (d >= DIM) {
        c.first[d] = 0;
        c.cnt[d] = 1;
        continue;
      }
      c.first[d] = (col >> d) & 1;
      c.cnt[d] = c.first[d] <= n - 1 ? (n - 1 - c.first[d]) / 2 + 1 : 0;
      c.n_cells *= c.cnt[d];
    }
    if (c.n_cells == 0) continue;
    PMG_TRY(ML::apply(pr->p, c, pr->arena, s));
  }
  return PMG_OK;
}

template <typename T, typename S>
MetricSmoothArgs<T, S> metric_args(pmg_problem *pr, int hl) {
  MetricSmoothArgs<T, S> a{};
  for (int l = 0; l < pr->nplev(); ++l) {
    a.lev[l].qt = qtab<T>(pr, l);
    a.lev[l].Tp = pr->pd<T>().tabs.Tp[l];
    a.lev[l].TpT = pr->pd<T>().tabs.TpT[l];
    a.lev[l].G = metric_of<S>(pr, hl, l);
    a.lev[l].invD = invd_of<S>(pr, hl, l);
  }
  a.n = pr->sizes[hl];
  a.full = pr->cfg.local_solver == PMG_LOCAL_FULL_V;
  a.n_iter = pr->cfg.n_local_iter;
  return a;
}

template <int DIM, typename T, typename S>
int metric_smooth_dim(pmg_problem *pr, int hl, int dir, T *u, const T *b, hipStream_t s) {
  MetricSmoothArgs<T, S> base = metric_args<T, S>(pr, hl);
  base.u = u;
  base.b = b;
  const int n = pr->sizes[hl], ncol = 1 << DIM;
  for (int ci = 0; ci < ncol; ++ci) {
    const int col = dir > 0 ? ci : ncol - 1 - ci;
    MetricSmoothArgs<T, S> a = base;
    a.n_patch = 1;
    for (int d = 0; d < 3; ++d) {
      if (d >= DIM) {
        a.first[d] = 0;
        a.cnt[d] = 1;
        continue;
      }
      a.first[d] = (col >> d) & 1 ? 1 : 2;
      a.cnt[d] = a.first[d] <= n - 1 ? (n - 1 - a.first[d]) / 2 + 1 : 0;
      a.n_patch *= a.cnt[d];
    }
    if (a.n_patch == 0) continue;
    PMG_TRY((MetricLaunchers<DIM, T, S>::smooth(pr->p, a, pr->arena, s)));
  }
  return PMG_OK;
}

template <int DIM, typename T, typename S>
int metric_local_dim(pmg_problem *pr, int hl, int first, int nb, const T *r, T *d, hipStream_t s) {
  MetricSmoothArgs<T, S> a = metric_args<T, S>(pr, hl);
  a.r_blocks = r;
  a.d_blocks = d;
  a.first_patch = first;
  PMG_TRY((MetricLaunchers<DIM, T, S>::local(pr->p, a, nb, pr->arena, s)));
  return PMG_OK;
}

// runtime (dimension, storage) -> instantiated metric launchers; 2D and FP64 ignore ST_BF16
#define PMG_METRIC_DISPATCH(FN, T, store, ...)                                     \
  do {                                                                             \
    if (pr->dim == 3) {                                                            \
      if constexpr (std::is_same<T, float>::value)                                 \
        if (store == ST_BF16) return FN<3, float, bf16>(__VA_ARGS__);              \
      return FN<3, T, T>(__VA_ARGS__);                                             \
    }                                                                              \
    return FN<2, T, T>(__VA_ARGS__);                                               \
  } while (0)

template <typename T>
int general_apply(pmg_problem *pr, int hl, bool resid, const T *b, const T *u, T *out, hipStream_t s, int store) {
  PMG_METRIC_DISPATCH(metric_apply_dim, T, store, pr, hl, resid, b, u, out, s);
}

template <typename T>
int general_smooth(pmg_problem *pr, int hl, int dir, T *u, const T *b, hipStream_t s, int store) {
  PMG_METRIC_DISPATCH(metric_smooth_dim, T, store, pr, hl, dir, u, b, s);
}

template <typename T>
int general_local(pmg_problem *pr, int hl, int first, int nb, const T *r, T *d, hipStream_t s, int store) {
  PMG_METRIC_DISPATCH(metric_local_dim, T, store, pr, hl, first, nb, r, d, s);
}

template <typename T>
int do_apply(pmg_problem *pr, int l, bool resid, const T *b, const T *u, T *out, hipStream_t s, int store = ST_NATIVE,
             bool mass = false) {
  if (pr->general) {
    if (mass) return fail(PMG_ERR_UNSUPPORTED, "the mass matrix is applied on the Cartesian mesh only");
    return general_apply<T>(pr, l, resid, b, u, out, s, store);
  }
  const int tc = tile_cells(pr->p);
  ApplyArgs<T> a{};
  a.Kt = pr->pd<T>().tabs.Kt;
  a.Mt = pr->pd<T>().tabs.Mt;
  // Laplacian: h^(d-2) sum_k K_k (x) M_others of the unit-interval matrices; mass: h^d
  a.c = mass ? (T)std::pow(1.0 / pr->sizes[l], pr->dim) : (T)pr->cscale(l);
  a.n = pr->sizes[l];
  a.ntile = (a.n + tc - 1) / tc;
  a.n_tiles = pr->dim == 3 ? a.ntile * a.ntile * a.ntile : a.ntile * a.ntile;
  a.u = u;
  a.b = b;
  a.out = out;
  PMG_TRY(launch_apply<T>(pr->dim, pr->p, mass ? 2 : (resid ? 1 : 0), a, pr->arena, s));
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
  a.direct = pr->cfg.local_solver == PMG_LOCAL_DIRECT;
  a.reinf = pr->cfg.local_smoother == PMG_SMOOTHER_REINFORCED;
  for (int l = 0; l < pr->nplev() && l < 4; ++l) a.om.w[l] = (T)pr->tab.omega[l];
  return a;
}

template <typename T>
int do_smooth(pmg_problem *pr, int l, int dir, T *u, const T *b, hipStream_t s, int store = ST_NATIVE) {
  if (pr->general) return general_smooth<T>(pr, l, dir, u, b, s, store);
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

// Work buffers of one V-cycle in precision T (r, z on levels below the finest, t on every
// level above the coarsest, the intermediates of the 1D transfer passes and the coarse
// solve's work vectors): the problem's own, or carved out of the static scratch array.
template <typename T>
struct VWork {
  static constexpr int kMaxLevels = 16;
  T *r[kMaxLevels] = {}, *z[kMaxLevels] = {}, *t[kMaxLevels] = {};
  T *tw1 = nullptr, *tw2 = nullptr;
  double *cw1 = nullptr, *cw2 = nullptr, *cwork = nullptr;
};

template <typename T>
VWork<T> own_work(pmg_problem *pr) {
  VWork<T> w;
  PrecData<T> &d = pr->pd<T>();
  for (size_t l = 0; l < pr->sizes.size(); ++l) {
    w.r[l] = d.r[l];
    w.z[l] = d.z[l];
    w.t[l] = d.t[l];
  }
  w.tw1 = d.tw1;
  w.tw2 = d.tw2;
  w.cw1 = pr->cw1;
  w.cw2 = pr->cw2;
  w.cwork = pr->cwork;
  return w;
}

template <typename T>
int do_restrict(pmg_problem *pr, int l, const T *fine, T *coarse, hipStream_t s, T *zero, T *tw1, T *tw2) {
  TransferArgs<T> a{};
  a.zero = zero;
  a.W1 = pr->pd<T>().tabs.W1;
  a.Wr = pr->pd<T>().tabs.Wr;
  a.nc = pr->sizes[l - 1];
  a.in = fine;
  a.out = coarse;
  a.w1 = tw1;
  a.w2 = tw2;
  PMG_TRY(launch_restrict<T>(pr->dim, pr->p, a, s));
  return PMG_OK;
}

template <typename T>
int do_prolong(pmg_problem *pr, int l, const T *coarse, T *fine, hipStream_t s, T *tw1, T *tw2) {
  TransferArgs<T> a{};
  a.W1 = pr->pd<T>().tabs.W1;
  a.Wr = pr->pd<T>().tabs.Wr;
  a.nc = pr->sizes[l - 1];
  a.in = coarse;
  a.out = fine;
  a.w1 = tw1;
  a.w2 = tw2;
  PMG_TRY(launch_prolong_add<T>(pr->dim, pr->p, a, s));
  return PMG_OK;
}

template <typename T>
int do_coarse(pmg_problem *pr, const T *r, T *z, hipStream_t s, const VWork<T> &w) {
  if (pr->general) {
    PMG_TRY(launch_coarse_dense<T>(pr->dim, pr->coarse_mi, pr->coarse_mi + 2, pr->Ainv, r, z, w.cwork, s));
    return PMG_OK;
  }
  CoarseArgs<T> a{};
  a.S = pr->S0;
  a.lam = pr->lam0;
  a.c0inv = 1.0 / pr->cscale(0);
  a.m = pr->tab.m0;
  a.mt = pr->tab.m0 + 2;
  a.r = r;
  a.z = z;
  a.w1 = w.cw1;
  a.w2 = w.cw2;
  PMG_TRY(launch_coarse<T>(pr->dim, a, s));
  return PMG_OK;
}

// h-multigrid V(n_pre, n_post) from a zero guess on the finest level (Sec. 2).
template <typename T>
int do_vcycle(pmg_problem *pr, const VWork<T> &w, const T *r, T *z, hipStream_t s, int store = ST_NATIVE) {
  const int L = pr->finest();
  if (L == 0) return do_coarse<T>(pr, r, z, s, w);
  for (int l = L; l >= 1; --l) {
    const T *R = l == L ? r : w.r[l];
    T *Z = l == L ? z : w.z[l];
    const int m = pr->p * pr->sizes[l] + 1;
    // the coarser levels' zero initial guess is written by the restriction into them
    if (l == L) PMG_TRY(launch_init_z<T>(pr->dim, m, Z, R, s));
    for (int k = 0; k < pr->cfg.n_pre; ++k) {
      int rc = do_smooth<T>(pr, l, +1, Z, R, s, store);
      if (rc) return rc;
    }
    int rc = do_apply<T>(pr, l, true, R, Z, w.t[l], s, store);
    if (rc) return rc;
    rc = do_restrict<T>(pr, l, w.t[l], w.r[l - 1], s, l - 1 >= 1 ? w.z[l - 1] : nullptr, w.tw1, w.tw2);
    if (rc) return rc;
  }
  int rc = do_coarse<T>(pr, w.r[0], w.z[0], s, w);
  if (rc) return rc;
  for (int l = 1; l <= L; ++l) {
    const T *R = l == L ? r : w.r[l];
    T *Z = l == L ? z : w.z[l];
    rc = do_prolong<T>(pr, l, w.z[l - 1], Z, s, w.tw1, w.tw2);
    if (rc) return rc;
    for (int k = 0; k < pr->cfg.n_post; ++k) {
      rc = do_smooth<T>(pr, l, -1, Z, R, s, store);
      if (rc) return rc;
    }
  }
  return PMG_OK;
}

// z = V(r) in mg_prec with the given work sets; the FP32 cycle takes its copies of r and z
// on the finest level from r32/z32.
int vcycle_with(pmg_problem *pr, int mg_prec, const double *r, double *z, hipStream_t s, const VWork<double> &w64,
                const VWork<float> &w32, float *r32, float *z32) {
  if (mg_prec == PMG_FP64) return do_vcycle<double>(pr, w64, r, z, s);
  const long N = pr->nodes(pr->finest());
  PMG_TRY(launch_cast_d2f(r, r32, N, s));
  int rc = do_vcycle<float>(pr, w32, r32, z32, s, mg_prec == PMG_FP32_BF16 ? ST_BF16 : ST_NATIVE);
  if (rc) return rc;
  PMG_TRY(launch_cast_f2d(z32, z, N, s));
  return PMG_OK;
}

int vcycle_any(pmg_problem *pr, int mg_prec, const double *r, double *z, hipStream_t s) {
  const int L = pr->finest();
  return vcycle_with(pr, mg_prec, r, z, s, own_work<double>(pr), own_work<float>(pr), pr->d32.r[L], pr->d32.z[L]);
}

// Lays the work set of one V-cycle in precision T out from byte offset `off` of `base`
// (256-byte aligned pieces); with base == nullptr only the offsets are computed.  Returns
// the end offset.
template <typename T>
size_t carve_work(pmg_problem *pr, char *base, size_t off, VWork<T> &w) {
  auto take = [&](size_t bytes) -> char * {
    off = (off + 255) / 256 * 256;
    char *ptr = base ? base + off : nullptr;
    off += bytes;
    return ptr;
  };
  const int L = pr->finest();
  for (int l = 0; l <= L; ++l) {
    const size_t N = (size_t)pr->nodes(l);
    if (l < L) {
      w.r[l] = (T *)take(N * sizeof(T));
      w.z[l] = (T *)take(N * sizeof(T));
    }
    if (l >= 1) w.t[l] = (T *)take(N * sizeof(T));
  }
  if (L >= 1) {
    const size_t mf = (size_t)pr->p * pr->sizes[L] + 1, mc = (size_t)pr->p * pr->sizes[L - 1] + 1;
    const size_t tw = pr->dim == 3 ? mf * mf * mc : mf * mc;
    w.tw1 = (T *)take(tw * sizeof(T));
    w.tw2 = (T *)take(tw * sizeof(T));
  }
  if (pr->general) {
    const size_t mi = (size_t)pr->coarse_mi;
    w.cwork = (double *)take((pr->dim == 3 ? mi * mi * mi : mi * mi) * sizeof(double));
  } else {
    const size_t m0 = (size_t)pr->tab.m0, m0d = pr->dim == 3 ? m0 * m0 * m0 : m0 * m0;
    w.cw1 = (double *)take(m0d * sizeof(double));
    w.cw2 = (double *)take(m0d * sizeof(double));
  }
  return off;
}

// Byte layout of pmg_vcycle_noalloc's work memory in mg_prec (base == nullptr: sizes only).
size_t noalloc_layout(pmg_problem *pr, int mg_prec, char *base, VWork<double> &w64, VWork<float> &w32, float **r32,
                      float **z32) {
  if (mg_prec == PMG_FP64) return carve_work<double>(pr, base, 0, w64);
  const size_t N = (size_t)pr->nodes(pr->finest());
  size_t off = carve_work<float>(pr, base, 0, w32);
  off = (off + 255) / 256 * 256;
  *r32 = base ? (float *)(base + off) : nullptr;
  off += N * sizeof(float);
  off = (off + 255) / 256 * 256;
  *z32 = base ? (float *)(base + off) : nullptr;
  return off + N * sizeof(float);
}

template <typename T>
int dev_alloc(pmg_problem *pr, T **out, size_t count) {
  return dev_alloc_in(pr->allocs, out, count);
}

void release(pmg_problem *pr) {
  for (void *ptr : pr->allocs) (void)hipFree(ptr);
  pr->allocs.clear();
  if (pr->hscal) (void)hipHostFree(pr->hscal);
  pr->hscal = nullptr;
  pr->dev = false;
}

}  // namespace

int pmg::upload_qtabs(std::vector<void *> &allocs, const std::vector<int> &degrees,
                      std::vector<QTabDev<double>> &q64, std::vector<QTabDev<float>> &q32,
                      std::vector<const double *> &B64, std::vector<const double *> &Dn64) {
  const int L = (int)degrees.size();
  int rc = PMG_OK;
  q64.assign(L, QTabDev<double>{});
  q32.assign(L, QTabDev<float>{});
  B64.assign(L, nullptr);
  Dn64.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    const QTab t = make_qtab(degrees[l]);
    const int k = t.q + 1;
    dvec Dn((size_t)t.nq * k, 0.0);  // derivative of the nodal basis at the Gauss points
    for (int g = 0; g < t.nq; ++g)
      for (int a = 0; a < k; ++a) {
        double sum = 0.0;
        for (int h = 0; h < t.nq; ++h) sum += t.Dq[(size_t)g * t.nq + h] * t.B[(size_t)h * k + a];
        Dn[(size_t)g * k + a] = sum;
      }
    const dvec *parts[] = {&t.B, &t.BT, &t.Dq, &t.DqT, &t.Bpc, &t.Bpi, &t.BpiT, &t.Dqp, &t.DqpT, &Dn};
    std::vector<double> flat;
    std::vector<size_t> off;
    for (const dvec *v : parts) {
      off.push_back(flat.size());
      flat.insert(flat.end(), v->begin(), v->end());
      flat.resize((flat.size() + 31) / 32 * 32 + 32, 0.0);
    }
    double *d64;
    float *d32;
    if ((rc = dev_alloc_in(allocs, &d64, flat.size())) || (rc = dev_alloc_in(allocs, &d32, flat.size()))) return rc;
    std::vector<float> flat32(flat.begin(), flat.end());
    PMG_HIP(hipMemcpy(d64, flat.data(), flat.size() * sizeof(double), hipMemcpyHostToDevice));
    PMG_HIP(hipMemcpy(d32, flat32.data(), flat32.size() * sizeof(float), hipMemcpyHostToDevice));
    auto bind = [&](auto &q, auto *base) {
      q.B = base + off[0]; q.BT = base + off[1]; q.Dq = base + off[2]; q.DqT = base + off[3];
      q.Bpc = base + off[4]; q.Bpi = base + off[5]; q.BpiT = base + off[6]; q.Dqp = base + off[7];
      q.DqpT = base + off[8];
    };
    bind(q64[l], d64);
    bind(q32[l], d32);
    B64[l] = d64 + off[0];
    Dn64[l] = d64 + off[9];
  }
  return PMG_OK;
}

namespace {

// Device data of the general path: 1D Gauss-point tables per p-level, the metric of every
// (h-level, p-level) in FP64/FP32/BF16, per-patch inverse diagonals computed on the device
// from element diagonals, and the dense inverse of the coarsest interior operator.
int init_general(pmg_problem *pr) {
  const int L = pr->nplev(), nh = (int)pr->sizes.size(), dim = pr->dim;
  int rc = PMG_OK;
  std::vector<const double *> B64, Dn64;
  if ((rc = upload_qtabs(pr->allocs, pr->degrees, pr->qt64, pr->qt32, B64, Dn64))) return rc;
  const size_t nslot = (size_t)nh * L;
  pr->G64.assign(nslot, nullptr);
  pr->G32.assign(nslot, nullptr);
  pr->G16.assign(nslot, nullptr);
  pr->invD64.assign(nslot, nullptr);
  pr->invD32.assign(nslot, nullptr);
  pr->invD16.assign(nslot, nullptr);
  const int nc = metric_components(dim);
  dvec G;
  for (int hl = 0; hl < nh; ++hl)
    for (int l = 0; l < L; ++l) {
      const int q = pr->degrees[l], n = pr->sizes[hl];
      const dvec &a = pr->coef[(size_t)hl * L + l];
      if (!metric(dim, n, pr->verts[hl], q, a.empty() ? nullptr : a.data(), G))
        return fail(PMG_ERR_INVALID_ARG, "a cell of h-level %d has a non-positive Jacobian determinant", hl);
      const long npts = pr->cells(hl) * (dim == 3 ? (long)(q + 1) * (q + 1) * (q + 1) : (long)(q + 1) * (q + 1));
      const size_t ng = (size_t)npts * nc;
      double *g64;
      float *g32;
      bf16 *g16;
      if ((rc = dev_alloc(pr, &g64, ng)) || (rc = dev_alloc(pr, &g32, ng)) || (rc = dev_alloc(pr, &g16, ng)))
        return rc;
      PMG_HIP(hipMemcpy(g64, G.data(), ng * sizeof(double), hipMemcpyHostToDevice));
      PMG_TRY(launch_convert<float>(g64, g32, (long)ng, nullptr));
      PMG_TRY(launch_convert<bf16>(g64, g16, (long)ng, nullptr));
      const size_t slot = (size_t)hl * L + l;
      pr->G64[slot] = g64;
      pr->G32[slot] = g32;
      pr->G16[slot] = g16;
      // element diagonals -> per-patch inverse diagonals (damping folded in)
      const long kd = dim == 3 ? (long)(q + 1) * (q + 1) * (q + 1) : (long)(q + 1) * (q + 1);
      void *cd = nullptr;
      PMG_HIP(hipMalloc(&cd, (size_t)(pr->cells(hl) * kd) * sizeof(double)));
      const long e1 = 2 * q - 1, k1 = n - 1;
      const size_t ni = (size_t)(dim == 3 ? k1 * k1 * k1 * e1 * e1 * e1 : k1 * k1 * e1 * e1);
      double *i64;
      float *i32;
      bf16 *i16;
      if ((rc = dev_alloc(pr, &i64, ni + 1)) || (rc = dev_alloc(pr, &i32, ni + 1)) || (rc = dev_alloc(pr, &i16, ni + 1))) {
        (void)hipFree(cd);
        return rc;
      }
      const double om = l == 0 ? 1.0 : pr->tab.omega[l];
      int krc = launch_cell_diag(dim, q, pr->cells(hl), B64[l], Dn64[l], g64, (double *)cd, nullptr);
      if (!krc) krc = launch_patch_invdiag<double>(dim, q, n, om, (const double *)cd, i64, nullptr);
      if (!krc) krc = launch_patch_invdiag<float>(dim, q, n, om, (const double *)cd, i32, nullptr);
      if (!krc) krc = launch_patch_invdiag<bf16>(dim, q, n, om, (const double *)cd, i16, nullptr);
      const hipError_t se = hipDeviceSynchronize();
      (void)hipFree(cd);
      if (krc || se != hipSuccess) return fail(PMG_ERR_DEVICE, "diagonal setup failed: %s", hipGetErrorString(se));
      pr->invD64[slot] = i64;
      pr->invD32[slot] = i32;
      pr->invD16[slot] = i16;
    }
  // coarsest mesh: dense interior operator of degree p -> Cholesky -> inverse
  {
    const int n0 = pr->sizes[0], p = pr->p;
    const int mi = p * n0 - 1;
    const long m = dim == 3 ? (long)mi * mi * mi : (long)mi * mi;
    pr->coarse_mi = mi;
    const int q = p, l = L - 1;
    const dvec &a = pr->coef[(size_t)0 * L + l];
    if (!metric(dim, n0, pr->verts[0], q, a.empty() ? nullptr : a.data(), G))
      return fail(PMG_ERR_INVALID_ARG, "degenerate coarse cell");
    dvec A;
    interior_matrix(dim, n0, p, G, A);
    double *Af;
    if ((rc = dev_alloc(pr, &Af, (size_t)(m * m))) || (rc = dev_alloc(pr, &pr->Ainv, (size_t)(m * m))) ||
        (rc = dev_alloc(pr, &pr->cwork, (size_t)m)))
      return rc;
    PMG_HIP(hipMemcpy(Af, A.data(), (size_t)(m * m) * sizeof(double), hipMemcpyHostToDevice));
    PMG_HIP(hipMemset(pr->Ainv, 0, (size_t)(m * m) * sizeof(double)));
    PMG_TRY(launch_set_identity(pr->Ainv, (int)m, nullptr));
    hipsolverHandle_t hs;
    if (hipsolverCreate(&hs) != HIPSOLVER_STATUS_SUCCESS) return fail(PMG_ERR_DEVICE, "hipsolverCreate failed");
    int lwork = 0, info = -1;
    int *dinfo = nullptr;
    double *work = nullptr;
    bool okf = hipMalloc((void **)&dinfo, sizeof(int)) == hipSuccess;
    okf = okf && hipsolverDnDpotrf_bufferSize(hs, HIPBLAS_FILL_MODE_LOWER, (int)m, Af, (int)m, &lwork) ==
                     HIPSOLVER_STATUS_SUCCESS;
    okf = okf && hipMalloc((void **)&work, (size_t)(lwork > 0 ? lwork : 1) * sizeof(double)) == hipSuccess;
    okf = okf && hipsolverDnDpotrf(hs, HIPBLAS_FILL_MODE_LOWER, (int)m, Af, (int)m, work, lwork, dinfo) ==
                     HIPSOLVER_STATUS_SUCCESS;
    okf = okf && hipMemcpy(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess && info == 0;
    okf = okf && hipsolverDnDpotrs(hs, HIPBLAS_FILL_MODE_LOWER, (int)m, (int)m, Af, (int)m, pr->Ainv, (int)m, dinfo) ==
                     HIPSOLVER_STATUS_SUCCESS;
    okf = okf && hipMemcpy(&info, dinfo, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess && info == 0;
    okf = okf && hipDeviceSynchronize() == hipSuccess;
    if (work) (void)hipFree(work);
    if (dinfo) (void)hipFree(dinfo);
    hipsolverDestroy(hs);
    if (!okf) return fail(PMG_ERR_DEVICE, "coarse Cholesky factorization failed (info %d)", info);
  }
  return PMG_OK;
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
  cfg->patch_lanes = PMG_LANES_AUTO;
  cfg->local_smoother = PMG_SMOOTHER_JACOBI;
}

int pmg_setup_mesh(int dim, const int32_t *n_cells, int n_hlevels, const double *vertices, pmg_mesh **out) {
  if (!out || !n_cells) return fail(PMG_ERR_INVALID_ARG, "n_cells or out is NULL");
  if (dim != 2 && dim != 3) return fail(PMG_ERR_INVALID_ARG, "dim must be 2 or 3, got %d", dim);
  for (int d = 0; d < dim; ++d)
    if (n_cells[d] < 2 || n_cells[d] > 1024)
      return fail(PMG_ERR_INVALID_ARG, "n_cells[%d] must be in [2, 1024], got %d", d, n_cells[d]);
  for (int d = 1; d < dim; ++d)
    if (n_cells[d] != n_cells[0])
      return fail(PMG_ERR_UNSUPPORTED, "meshes with different cell counts per direction are not supported");
  const int n = n_cells[0];
  if (n_hlevels < 0) return fail(PMG_ERR_INVALID_ARG, "n_hlevels must be >= 0");
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
    if (vertices) {
      const size_t nv = dim == 3 ? (size_t)(n + 1) * (n + 1) * (n + 1) : (size_t)(n + 1) * (n + 1);
      m->verts.assign(vertices, vertices + nv * dim);
      for (double x : m->verts)
        if (!std::isfinite(x)) {
          delete m;
          return fail(PMG_ERR_INVALID_ARG, "vertex coordinates must be finite");
        }
    }
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
  if (c.local_solver != PMG_LOCAL_HALF_V && c.local_solver != PMG_LOCAL_FULL_V && c.local_solver != PMG_LOCAL_DIRECT)
    return fail(PMG_ERR_INVALID_ARG, "local_solver unknown");
  if (c.local_smoother != PMG_SMOOTHER_JACOBI && c.local_smoother != PMG_SMOOTHER_REINFORCED)
    return fail(PMG_ERR_INVALID_ARG, "local_smoother unknown");
  if (m->verts.size() && (c.local_solver == PMG_LOCAL_DIRECT || c.local_smoother == PMG_SMOOTHER_REINFORCED))
    return fail(PMG_ERR_UNSUPPORTED, "fast-diagonalization local solvers need the Cartesian path");
  if (c.n_local_iter < 1 || c.n_local_iter > 64) return fail(PMG_ERR_INVALID_ARG, "n_local_iter must be in [1, 64]");
  if (c.n_pre < 0 || c.n_post < 0 || c.n_pre > 16 || c.n_post > 16)
    return fail(PMG_ERR_INVALID_ARG, "n_pre and n_post must be in [0, 16]");
  if (c.max_iter < 1) return fail(PMG_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (!(c.rtol > 0.0) || !(c.rtol < 1.0)) return fail(PMG_ERR_INVALID_ARG, "rtol must be in (0, 1)");
  if (c.n_omega < 0 || c.n_omega > (int)deg.size()) return fail(PMG_ERR_INVALID_ARG, "n_omega out of range");
  if (c.patch_lanes != PMG_LANES_AUTO && c.patch_lanes != PMG_LANES_NARROW && c.patch_lanes != PMG_LANES_WIDE &&
      c.patch_lanes != PMG_LANES_HALF)
    return fail(PMG_ERR_INVALID_ARG, "patch_lanes unknown");
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
    if (c.n_omega > 0)
      om.assign(c.omega, c.omega + c.n_omega);
    else if (c.local_smoother == PMG_SMOOTHER_REINFORCED)
      om.assign(deg.size(), 1.0);  // the reinforced preconditioner is exact on Cartesian patches
    build_tables(pr->dim, degree, deg, om, pr->sizes[0], pr->tab);
    pr->general = !m->verts.empty();
    for (int l : pr->sizes)
      pr->verts.push_back(m->verts.empty() ? cartesian_vertices(pr->dim, l)
                                           : level_vertices(pr->dim, m->n, m->verts, l));
    pr->coef.assign(pr->sizes.size() * deg.size(), dvec());
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

int pmg_get_qpoints(const pmg_problem *pr, int hlevel, int plevel, double *xyz) {
  if (!pr || !xyz) return fail(PMG_ERR_INVALID_ARG, "problem or xyz is NULL");
  if (int rc = check_level(pr, hlevel)) return rc;
  if (plevel < 0 || plevel >= (int)pr->degrees.size()) return fail(PMG_ERR_INVALID_ARG, "plevel out of range");
  dvec out;
  gauss_points(pr->dim, pr->sizes[hlevel], pr->verts[hlevel], pr->degrees[plevel], out);
  std::memcpy(xyz, out.data(), out.size() * sizeof(double));
  return PMG_OK;
}

int pmg_set_coefficient(pmg_problem *pr, int hlevel, int plevel, const double *a_q) {
  if (!pr) return fail(PMG_ERR_INVALID_ARG, "problem is NULL");
  if (pr->dev) return fail(PMG_ERR_STATE, "coefficients must be set before pmg_device_init");
  if (int rc = check_level(pr, hlevel)) return rc;
  if (plevel < 0 || plevel >= (int)pr->degrees.size()) return fail(PMG_ERR_INVALID_ARG, "plevel out of range");
  const int q = pr->degrees[plevel];
  const size_t npts = (size_t)pr->cells(hlevel) * (pr->dim == 3 ? (size_t)(q + 1) * (q + 1) * (q + 1) : (size_t)(q + 1) * (q + 1));
  dvec &dst = pr->coef[(size_t)hlevel * pr->degrees.size() + plevel];
  if (!a_q) {
    dst.clear();
    return PMG_OK;
  }
  for (size_t i = 0; i < npts; ++i)
    if (!(a_q[i] > 0.0) || !std::isfinite(a_q[i])) return fail(PMG_ERR_INVALID_ARG, "coefficient must be positive and finite");
  dst.assign(a_q, a_q + npts);
  return PMG_OK;
}

int pmg_device_init(pmg_problem *pr) {
  if (!pr) return fail(PMG_ERR_INVALID_ARG, "problem is NULL");
  if (pr->dev) return PMG_OK;
  PMG_HIP(hipGetDevice(&pr->device));
  int lds = 0, ncu = 0;
  PMG_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, pr->device));
  PMG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pr->device));
  if (int rc = resolve_scratch(pr->device)) return rc;
  pr->arena.lds_max = (size_t)lds;
  pr->arena.ncu = ncu > 0 ? ncu : 256;
  pr->arena.patch_lanes = pr->cfg.patch_lanes;
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
  pr->general = pr->general || [&]() {
    for (const dvec &a : pr->coef)
      if (!a.empty()) return true;
    return false;
  }();
  if (pr->general && pr->hcode != 0) return bail(fail(PMG_ERR_UNSUPPORTED, "the general path compiles the paper's p-hierarchy only"));
  if (pr->general && (pr->cfg.local_solver == PMG_LOCAL_DIRECT || pr->cfg.local_smoother == PMG_SMOOTHER_REINFORCED))
    return bail(fail(PMG_ERR_UNSUPPORTED, "fast-diagonalization local solvers need the Cartesian path"));
  size_t need = 0;
  for (int prec = 0; prec < 2; ++prec) {
    size_t b1 = pr->general ? metric_patch_arena_bytes(pr->dim, prec, pr->p) : patch_arena_bytes(pr->dim, prec, pr->p, pr->hcode);
    size_t b2 = pr->general ? metric_apply_arena_bytes(pr->dim, prec, pr->p) : apply_arena_bytes(pr->dim, prec, pr->p);
    if (b1 > pr->arena.lds_max && b1 > need) need = b1;
    if (b2 > pr->arena.lds_max && b2 > need) need = b2;
  }
  if (need) {
    pr->arena.slots = 2 * (ncu > 0 ? ncu : 256);
    void *g = nullptr;
    if ((rc = dev_alloc(pr, (unsigned char **)&g, need * pr->arena.slots))) return bail(rc);
    pr->arena.global = g;
  }
  if (pr->general && (rc = init_general(pr))) return bail(rc);
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
  return do_apply<float>(pr, hlevel, false, nullptr, (const float *)u, (float *)v, s, store_of(prec));
}

int pmg_mass_operator(pmg_problem *pr, int hlevel, int prec, const void *u, void *v, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (!u || !v) return fail(PMG_ERR_INVALID_ARG, "u or v is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64)
    return do_apply<double>(pr, hlevel, false, nullptr, (const double *)u, (double *)v, s, ST_NATIVE, true);
  return do_apply<float>(pr, hlevel, false, nullptr, (const float *)u, (float *)v, s, store_of(prec), true);
}

int pmg_residual(pmg_problem *pr, int hlevel, int prec, const void *b, const void *u, void *r, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (!u || !b || !r) return fail(PMG_ERR_INVALID_ARG, "b, u or r is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return do_apply<double>(pr, hlevel, true, (const double *)b, (const double *)u, (double *)r, s);
  return do_apply<float>(pr, hlevel, true, (const float *)b, (const float *)u, (float *)r, s, store_of(prec));
}

int pmg_smooth(pmg_problem *pr, int hlevel, int prec, int color_dir, void *u, const void *b, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (color_dir != 1 && color_dir != -1) return fail(PMG_ERR_INVALID_ARG, "color_dir must be +1 or -1");
  if (!u || !b) return fail(PMG_ERR_INVALID_ARG, "u or b is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return do_smooth<double>(pr, hlevel, color_dir, (double *)u, (const double *)b, s);
  return do_smooth<float>(pr, hlevel, color_dir, (float *)u, (const float *)b, s, store_of(prec));
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
  if (pr->general) {
    if (prec == PMG_FP64) return general_local<double>(pr, hlevel, first_patch, n_patches, (const double *)r, (double *)d, s, ST_NATIVE);
    return general_local<float>(pr, hlevel, first_patch, n_patches, (const float *)r, (float *)d, s, store_of(prec));
  }
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
  if (prec == PMG_FP64)
    return do_restrict<double>(pr, hlevel, (const double *)fine, (double *)coarse, s, nullptr, pr->d64.tw1, pr->d64.tw2);
  return do_restrict<float>(pr, hlevel, (const float *)fine, (float *)coarse, s, nullptr, pr->d32.tw1, pr->d32.tw2);
}

int pmg_prolongate_add(pmg_problem *pr, int hlevel, int prec, const void *coarse, void *fine, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_level(pr, hlevel)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (hlevel < 1) return fail(PMG_ERR_INVALID_ARG, "prolongation needs hlevel >= 1");
  if (!fine || !coarse) return fail(PMG_ERR_INVALID_ARG, "fine or coarse is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64)
    return do_prolong<double>(pr, hlevel, (const double *)coarse, (double *)fine, s, pr->d64.tw1, pr->d64.tw2);
  return do_prolong<float>(pr, hlevel, (const float *)coarse, (float *)fine, s, pr->d32.tw1, pr->d32.tw2);
}

int pmg_coarse_solve(pmg_problem *pr, int prec, const void *r, void *z, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_prec(prec)) return rc;
  if (!r || !z) return fail(PMG_ERR_INVALID_ARG, "r or z is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return do_coarse<double>(pr, (const double *)r, (double *)z, s, own_work<double>(pr));
  return do_coarse<float>(pr, (const float *)r, (float *)z, s, own_work<float>(pr));
}

int pmg_vcycle(pmg_problem *pr, int mg_prec, const double *r, double *z, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_prec(mg_prec)) return rc;
  if (!r || !z) return fail(PMG_ERR_INVALID_ARG, "r or z is NULL");
  return vcycle_any(pr, mg_prec, r, z, (hipStream_t)stream);
}

int pmg_vcycle_noalloc(pmg_problem *pr, int mg_prec, const double *r, double *z, void *stream) {
  if (int rc = check_ready(pr)) return rc;
  if (int rc = check_prec(mg_prec)) return rc;
  if (!r || !z) return fail(PMG_ERR_INVALID_ARG, "r or z is NULL");
  if (pr->arena.global)
    return fail(PMG_ERR_UNSUPPORTED, "this problem's kernels need a workgroup arena in global memory");
  int device = -1;
  PMG_HIP(hipGetDevice(&device));
  if (device != pr->device)
    return fail(PMG_ERR_INVALID_ARG, "the problem lives on device %d but device %d is current", pr->device, device);
  char *base = scratch_of(device);
  if (!base) return fail(PMG_ERR_STATE, "the scratch array of device %d is not resolved", device);
  VWork<double> w64;
  VWork<float> w32;
  float *r32 = nullptr, *z32 = nullptr;
  const size_t need = noalloc_layout(pr, mg_prec, nullptr, w64, w32, &r32, &z32);
  if (need > (size_t)PMG_NOALLOC_SCRATCH_BYTES)
    return fail(PMG_ERR_INVALID_ARG, "the V-cycle needs %zu bytes of work memory, above the %zu of the scratch array",
                need, (size_t)PMG_NOALLOC_SCRATCH_BYTES);
  noalloc_layout(pr, mg_prec, base, w64, w32, &r32, &z32);
  return vcycle_with(pr, mg_prec, r, z, (hipStream_t)stream, w64, w32, r32, z32);
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
