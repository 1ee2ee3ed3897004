// C interface of general hex meshes with stored maps: setup (host), device data, the
// operator apply / residual and the colored patch smoother through the stored maps.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "hex_launch.h"
#include "hex_setup.h"
#include "launch.h"
#include "pmg.h"
#include "problem.h"
#include "tab_layout.h"

using namespace pmg;

struct pmg_hex {
  HexHost h;
  std::vector<int> degrees;
  pmg_config cfg{};
  Tables tab;
  // device state
  bool dev = false;
  int device = -1;
  std::vector<void *> allocs;
  DevTabs<double> t64{};
  DevTabs<float> t32{};
  std::vector<QTabDev<double>> qt64;
  std::vector<QTabDev<float>> qt32;
  std::vector<const double *> G64, invD64;
  std::vector<const float *> G32, invD32;
  int32_t *plist = nullptr, *pmap = nullptr, *pcells = nullptr, *clist = nullptr, *cdof = nullptr;
  unsigned char *bnd = nullptr;
  Arena arena;
  int nplev() const { return (int)degrees.size(); }
};

namespace {

void release(pmg_hex *hx) {
  for (void *p : hx->allocs) (void)hipFree(p);
  hx->allocs.clear();
  hx->dev = false;
}

int check_ready(const pmg_hex *hx) {
  if (!hx) return fail(PMG_ERR_INVALID_ARG, "hex problem is NULL");
  if (!hx->dev) return fail(PMG_ERR_STATE, "pmg_hex_device_init has not been called");
  return PMG_OK;
}

template <typename T>
struct Sel;
template <>
struct Sel<double> {
  static const DevTabs<double> &tabs(const pmg_hex *h) { return h->t64; }
  static const QTabDev<double> &qt(const pmg_hex *h, int l) { return h->qt64[l]; }
  static const double *G(const pmg_hex *h, int l) { return h->G64[l]; }
  static const double *invD(const pmg_hex *h, int l) { return h->invD64[l]; }
};
template <>
struct Sel<float> {
  static const DevTabs<float> &tabs(const pmg_hex *h) { return h->t32; }
  static const QTabDev<float> &qt(const pmg_hex *h, int l) { return h->qt32[l]; }
  static const float *G(const pmg_hex *h, int l) { return h->G32[l]; }
  static const float *invD(const pmg_hex *h, int l) { return h->invD32[l]; }
};

template <int DIM, typename T>
int hex_apply_dim(pmg_hex *hx, bool resid, const T *b, const T *u, T *out, hipStream_t s) {
  using HL = HexLaunchers<DIM, T>;
  const HexHost &h = hx->h;
  const int L = hx->nplev();
  PMG_TRY(HL::apply_init(h.n_dofs, resid, hx->bnd, b, u, out, s));
  MetricApplyArgs<T, T> a{};
  a.qt = Sel<T>::qt(hx, L - 1);
  a.G = Sel<T>::G(hx, L - 1);
  a.sign = resid ? T(-1) : T(1);
  a.u = u;
  a.out = out;
  a.cdof = hx->cdof;
  a.bnd = hx->bnd;
  const int ncol = (int)h.cfirst.size() - 1;
  for (int c = 0; c < ncol; ++c) {
    a.clist = hx->clist + h.cfirst[c];
    a.n_cells = h.cfirst[c + 1] - h.cfirst[c];
    PMG_TRY(HL::apply(h.p, a, hx->arena, s));
  }
  return PMG_OK;
}

template <int DIM, typename T>
int hex_smooth_dim(pmg_hex *hx, int dir, T *u, const T *b, hipStream_t s) {
  const HexHost &h = hx->h;
  MetricSmoothArgs<T, T> a{};
  for (int l = 0; l < hx->nplev(); ++l) {
    a.lev[l].qt = Sel<T>::qt(hx, l);
    a.lev[l].Tp = Sel<T>::tabs(hx).Tp[l];
    a.lev[l].TpT = Sel<T>::tabs(hx).TpT[l];
    a.lev[l].G = Sel<T>::G(hx, l);
    a.lev[l].invD = Sel<T>::invD(hx, l);
  }
  a.full = hx->cfg.local_solver == PMG_LOCAL_FULL_V;
  a.n_iter = hx->cfg.n_local_iter;
  a.u = u;
  a.b = b;
  a.pmap = hx->pmap;
  a.pcells = hx->pcells;
  const int ncol = (int)h.pfirst.size() - 1;
  for (int ci = 0; ci < ncol; ++ci) {
    const int c = dir > 0 ? ci : ncol - 1 - ci;
    a.plist = hx->plist + h.pfirst[c];
    a.n_patch = h.pfirst[c + 1] - h.pfirst[c];
    if (a.n_patch == 0) continue;
    PMG_TRY((HexLaunchers<DIM, T>::smooth(h.p, a, hx->arena, s)));
  }
  return PMG_OK;
}

template <typename T>
int hex_apply(pmg_hex *hx, bool resid, const T *b, const T *u, T *out, hipStream_t s) {
  return hx->h.dim == 3 ? hex_apply_dim<3, T>(hx, resid, b, u, out, s) : hex_apply_dim<2, T>(hx, resid, b, u, out, s);
}

template <typename T>
int hex_smooth(pmg_hex *hx, int dir, T *u, const T *b, hipStream_t s) {
  return hx->h.dim == 3 ? hex_smooth_dim<3, T>(hx, dir, u, b, s) : hex_smooth_dim<2, T>(hx, dir, u, b, s);
}

template <typename T>
int upload(pmg_hex *hx, T **dst, const std::vector<T> &src) {
  if (int rc = dev_alloc_in(hx->allocs, dst, src.size() ? src.size() : 1)) return rc;
  if (!src.empty()) PMG_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return PMG_OK;
}

// metric, element diagonals and per-patch inverse diagonals of every p-level
int init_levels(pmg_hex *hx) {
  const HexHost &h = hx->h;
  const int dim = h.dim, L = hx->nplev(), ncn = 1 << dim;
  std::vector<const double *> B64, Dn64;
  int rc = PMG_OK;
  if ((rc = upload_qtabs(hx->allocs, hx->degrees, hx->qt64, hx->qt32, B64, Dn64))) return rc;
  hx->G64.assign(L, nullptr);
  hx->G32.assign(L, nullptr);
  hx->invD64.assign(L, nullptr);
  hx->invD32.assign(L, nullptr);
  const long np = (long)h.pvert.size();
  dvec G;
  for (int l = 0; l < L; ++l) {
    const int q = hx->degrees[l];
    auto corners = [&](long c, double X[8][3]) {
      for (int j = 0; j < ncn; ++j)
        for (int a = 0; a < dim; ++a) X[j][a] = h.xyz[(size_t)h.cverts[(size_t)c * ncn + j] * dim + a];
    };
    if (!metric_cells(dim, h.n_cells, corners, q, nullptr, G))
      return fail(PMG_ERR_INVALID_ARG, "a cell has a non-positive Jacobian determinant at a Gauss point");
    const size_t ng = G.size();
    double *g64;
    float *g32;
    if ((rc = dev_alloc_in(hx->allocs, &g64, ng)) || (rc = dev_alloc_in(hx->allocs, &g32, ng))) return rc;
    PMG_HIP(hipMemcpy(g64, G.data(), ng * sizeof(double), hipMemcpyHostToDevice));
    PMG_TRY(launch_convert<float>(g64, g32, (long)ng, nullptr));
    hx->G64[l] = g64;
    hx->G32[l] = g32;
    const long kd = dim == 3 ? (long)(q + 1) * (q + 1) * (q + 1) : (long)(q + 1) * (q + 1);
    const long e1 = 2 * q - 1, nip = dim == 3 ? e1 * e1 * e1 : e1 * e1;
    double *i64;
    float *i32;
    if ((rc = dev_alloc_in(hx->allocs, &i64, (size_t)(np * nip + 1))) ||
        (rc = dev_alloc_in(hx->allocs, &i32, (size_t)(np * nip + 1))))
      return rc;
    double *cd = nullptr;  // element diagonals: setup only
    PMG_HIP(hipMalloc((void **)&cd, (size_t)(h.n_cells * kd) * sizeof(double)));
    const double om = l == 0 ? 1.0 : hx->tab.omega[l];
    int krc = launch_cell_diag(dim, q, h.n_cells, B64[l], Dn64[l], g64, cd, nullptr);
    if (!krc) krc = launch_patch_invdiag_list<double>(dim, q, np, hx->pcells, om, cd, i64, nullptr);
    if (!krc) krc = launch_patch_invdiag_list<float>(dim, q, np, hx->pcells, om, cd, i32, nullptr);
    const hipError_t se = hipDeviceSynchronize();
    (void)hipFree(cd);
    if (krc || se != hipSuccess) return fail(PMG_ERR_DEVICE, "diagonal setup failed: %s", hipGetErrorString(se));
    hx->invD64[l] = i64;
    hx->invD32[l] = i32;
  }
  return PMG_OK;
}

}  // namespace

extern "C" {

int pmg_setup_hex(int dim, int degree, int64_t n_vertices, const double *vertices, int64_t n_cells,
                  const int32_t *cell_vertices, int64_t n_dofs, const int32_t *cell_dofs, const pmg_config *cfg,
                  pmg_hex **out) {
  if (!out || !vertices || !cell_vertices || !cell_dofs)
    return fail(PMG_ERR_INVALID_ARG, "out, vertices, cell_vertices or cell_dofs is NULL");
  pmg_config c;
  pmg_default_config(&c);
  if (cfg) c = *cfg;
  if (c.local_solver != PMG_LOCAL_HALF_V && c.local_solver != PMG_LOCAL_FULL_V)
    return fail(c.local_solver == PMG_LOCAL_DIRECT ? PMG_ERR_UNSUPPORTED : PMG_ERR_INVALID_ARG,
                "local_solver must be PMG_LOCAL_HALF_V or PMG_LOCAL_FULL_V on general meshes");
  if (c.local_smoother != PMG_SMOOTHER_JACOBI)
    return fail(PMG_ERR_UNSUPPORTED, "general meshes use the Jacobi local smoother");
  if (c.n_local_iter < 1 || c.n_local_iter > 64) return fail(PMG_ERR_INVALID_ARG, "n_local_iter must be in [1, 64]");
  if (degree < 1 || degree > 8) return fail(PMG_ERR_INVALID_ARG, "degree must be in [1, 8], got %d", degree);
  std::vector<int> deg;
  for (int x = 1; x < degree; x = 2 * x + 1) deg.push_back(x);
  deg.push_back(degree);
  if (c.n_omega < 0 || c.n_omega > (int)deg.size()) return fail(PMG_ERR_INVALID_ARG, "n_omega out of range");
  for (int i = 1; i < c.n_omega; ++i)
    if (!(c.omega[i] > 0.0 && c.omega[i] < 2.0)) return fail(PMG_ERR_INVALID_ARG, "omega[%d] must be in (0, 2)", i);
  try {
    pmg_hex *hx = new pmg_hex;
    std::string err;
    const int rc = hex_build(dim, degree, (long)n_vertices, vertices, (long)n_cells, cell_vertices, (long)n_dofs,
                             cell_dofs, hx->h, err);
    if (rc) {
      delete hx;
      return fail(rc, "%s", err.c_str());
    }
    hx->degrees = deg;
    hx->cfg = c;
    dvec om;
    if (c.n_omega > 0) om.assign(c.omega, c.omega + c.n_omega);
    build_tables(dim, degree, deg, om, 2, hx->tab);
    *out = hx;
  } catch (const std::exception &e) {
    return fail(PMG_ERR_INVALID_ARG, "setup failed: %s", e.what());
  }
  return PMG_OK;
}

int pmg_hex_sizes(const pmg_hex *hx, int64_t *n_patches, int *n_patch_colors, int *n_cell_colors, int *n_plevels,
                  int32_t *degrees, double *omega) {
  if (!hx) return fail(PMG_ERR_INVALID_ARG, "hex problem is NULL");
  if (n_patches) *n_patches = (int64_t)hx->h.pvert.size();
  if (n_patch_colors) *n_patch_colors = (int)hx->h.pfirst.size() - 1;
  if (n_cell_colors) *n_cell_colors = (int)hx->h.cfirst.size() - 1;
  if (n_plevels) *n_plevels = hx->nplev();
  for (int i = 0; i < hx->nplev(); ++i) {
    if (degrees) degrees[i] = hx->degrees[i];
    if (omega) omega[i] = hx->tab.omega[i];
  }
  return PMG_OK;
}

int pmg_hex_export(const pmg_hex *hx, int32_t *patch_vertex, int32_t *patch_color, int32_t *patch_cells,
                   int32_t *patch_closure, int32_t *cell_color, uint8_t *boundary) {
  if (!hx) return fail(PMG_ERR_INVALID_ARG, "hex problem is NULL");
  const HexHost &h = hx->h;
  auto put = [](auto *dst, const auto &src) {
    if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(src[0]));
  };
  put(patch_vertex, h.pvert);
  put(patch_color, h.pcolor);
  put(patch_cells, h.pcells);
  put(patch_closure, h.pmap);
  put(cell_color, h.ccolor);
  put(boundary, h.bnd);
  return PMG_OK;
}

int pmg_hex_device_init(pmg_hex *hx) {
  if (!hx) return fail(PMG_ERR_INVALID_ARG, "hex problem is NULL");
  if (hx->dev) return PMG_OK;
  PMG_HIP(hipGetDevice(&hx->device));
  int lds = 0, ncu = 0;
  PMG_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hx->device));
  PMG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, hx->device));
  hx->arena.lds_max = (size_t)lds;
  hx->arena.ncu = ncu > 0 ? ncu : 256;
  int rc = PMG_OK;
  auto bail = [&](int code) {
    release(hx);
    return code;
  };
  const HexHost &h = hx->h;
  std::vector<double> flat;
  std::vector<size_t> off;
  flatten_tabs(hx->tab, flat, off);
  double *t64 = nullptr;
  float *t32 = nullptr;
  if ((rc = dev_alloc_in(hx->allocs, &t64, flat.size())) || (rc = dev_alloc_in(hx->allocs, &t32, flat.size())))
    return bail(rc);
  std::vector<float> flat32(flat.begin(), flat.end());
  if (hipMemcpy(t64, flat.data(), flat.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t32, flat32.data(), flat32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(PMG_ERR_DEVICE, "table upload failed"));
  bind_tabs(hx->t64, hx->tab, t64, off);
  bind_tabs(hx->t32, hx->tab, t32, off);
  std::vector<unsigned char> bnd(h.bnd.begin(), h.bnd.end());
  if ((rc = upload(hx, &hx->plist, h.plist)) || (rc = upload(hx, &hx->pmap, h.pmap)) ||
      (rc = upload(hx, &hx->pcells, h.pcells)) || (rc = upload(hx, &hx->clist, h.clist)) ||
      (rc = upload(hx, &hx->cdof, h.cdofs)) || (rc = upload(hx, &hx->bnd, bnd)))
    return bail(rc);
  // global arena for kernels whose workgroup arena exceeds the LDS limit
  size_t need = 0;
  for (int prec = 0; prec < 2; ++prec) {
    const int p = h.p;
    size_t b1, b2;
    if (h.dim == 3) {
      b1 = prec ? HexLaunchers<3, float>::patch_bytes(p) : HexLaunchers<3, double>::patch_bytes(p);
      b2 = prec ? HexLaunchers<3, float>::apply_bytes(p) : HexLaunchers<3, double>::apply_bytes(p);
    } else {
      b1 = prec ? HexLaunchers<2, float>::patch_bytes(p) : HexLaunchers<2, double>::patch_bytes(p);
      b2 = prec ? HexLaunchers<2, float>::apply_bytes(p) : HexLaunchers<2, double>::apply_bytes(p);
    }
    if (b1 > hx->arena.lds_max && b1 > need) need = b1;
    if (b2 > hx->arena.lds_max && b2 > need) need = b2;
  }
  if (need) {
    hx->arena.slots = 2 * hx->arena.ncu;
    unsigned char *g = nullptr;
    if ((rc = dev_alloc_in(hx->allocs, &g, need * hx->arena.slots))) return bail(rc);
    hx->arena.global = g;
  }
  if ((rc = init_levels(hx))) return bail(rc);
  hx->dev = true;
  return PMG_OK;
}

int pmg_hex_apply(pmg_hex *hx, int prec, const void *u, void *v, void *stream) {
  if (int rc = check_ready(hx)) return rc;
  if (prec != PMG_FP64 && prec != PMG_FP32) return fail(PMG_ERR_INVALID_ARG, "precision must be FP64 or FP32");
  if (!u || !v) return fail(PMG_ERR_INVALID_ARG, "u or v is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return hex_apply<double>(hx, false, nullptr, (const double *)u, (double *)v, s);
  return hex_apply<float>(hx, false, nullptr, (const float *)u, (float *)v, s);
}

int pmg_hex_residual(pmg_hex *hx, int prec, const void *b, const void *u, void *r, void *stream) {
  if (int rc = check_ready(hx)) return rc;
  if (prec != PMG_FP64 && prec != PMG_FP32) return fail(PMG_ERR_INVALID_ARG, "precision must be FP64 or FP32");
  if (!b || !u || !r) return fail(PMG_ERR_INVALID_ARG, "b, u or r is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return hex_apply<double>(hx, true, (const double *)b, (const double *)u, (double *)r, s);
  return hex_apply<float>(hx, true, (const float *)b, (const float *)u, (float *)r, s);
}

int pmg_hex_smooth(pmg_hex *hx, int prec, int color_dir, void *u, const void *b, void *stream) {
  if (int rc = check_ready(hx)) return rc;
  if (prec != PMG_FP64 && prec != PMG_FP32) return fail(PMG_ERR_INVALID_ARG, "precision must be FP64 or FP32");
  if (color_dir != 1 && color_dir != -1) return fail(PMG_ERR_INVALID_ARG, "color_dir must be +1 or -1");
  if (!u || !b) return fail(PMG_ERR_INVALID_ARG, "u or b is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (prec == PMG_FP64) return hex_smooth<double>(hx, color_dir, (double *)u, (const double *)b, s);
  return hex_smooth<float>(hx, color_dir, (float *)u, (const float *)b, s);
}

void pmg_hex_destroy(pmg_hex *hx) {
  if (!hx) return;
  release(hx);
  delete hx;
}

}  // extern "C"
