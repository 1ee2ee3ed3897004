// Internal state behind the opaque handles of the C interface (shared by the
// single-problem entry points and the batched ones).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>
#include <vector>

#include "geometry.h"
#include "host_tables.h"
#include "launch.h"
#include "pmg.h"

namespace pmg {

// Stores a formatted message for pmg_last_error (thread-local) and returns `code`.
int fail(int code, const char *fmt, ...);

#define PMG_TRY(expr)                                                        \
  do {                                                                       \
    int rc_ = (expr);                                                        \
    if (rc_ != 0) return ::pmg::fail(rc_ == -3 ? PMG_ERR_OUT_OF_MEMORY : PMG_ERR_DEVICE, "%s failed (%d): %s", #expr, rc_, \
                              hipGetErrorString(hipGetLastError()));         \
  } while (0)

#define PMG_HIP(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return ::pmg::fail(e_ == hipErrorOutOfMemory ? PMG_ERR_OUT_OF_MEMORY : PMG_ERR_DEVICE, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                                     \
  } while (0)

// hipMalloc of count elements (plus slack), recorded in allocs for release.
template <typename T>
int dev_alloc_in(std::vector<void *> &allocs, T **out, size_t count) {
  void *ptr = nullptr;
  PMG_HIP(hipMalloc(&ptr, count * sizeof(T) + 64));
  allocs.push_back(ptr);
  *out = reinterpret_cast<T *>(ptr);
  return 0;
}

// 1D Gauss-point tables of the metric path for every degree, in FP64 and FP32 on the
// device; B64/Dn64: the FP64 basis values and nodal-basis derivatives at the Gauss points.
int upload_qtabs(std::vector<void *> &allocs, const std::vector<int> &degrees, std::vector<QTabDev<double>> &q64,
                 std::vector<QTabDev<float>> &q32, std::vector<const double *> &B64, std::vector<const double *> &Dn64);

template <typename T>
struct PrecData {
  DevTabs<T> tabs{};
  std::vector<T *> r, z, t;   // per h-level work vectors
  T *tw1 = nullptr, *tw2 = nullptr;  // intermediates of the 1D transfer passes
};

}  // namespace pmg

struct pmg_mesh {
  int dim = 3, n = 0;
  std::vector<int> sizes;   // cells per direction, coarsest first
  std::vector<double> verts;  // finest-level vertices, empty for the Cartesian unit box
};

struct pmg_problem {
  int dim = 3, p = 1, hcode = 0;
  std::vector<int> sizes, degrees;
  pmg_config cfg{};
  pmg::Tables tab;
  // device state
  bool dev = false;
  int device = -1;
  std::vector<void *> allocs;
  pmg::PrecData<double> d64;
  pmg::PrecData<float> d32;
  double *S0 = nullptr, *lam0 = nullptr, *cw1 = nullptr, *cw2 = nullptr;
  double *fr[2] = {nullptr, nullptr}, *fz = nullptr, *fp = nullptr, *fq = nullptr;
  double *part = nullptr, *scal = nullptr, *hscal = nullptr;
  pmg::Arena arena;
  // general path (distorted vertices or a coefficient): per (h-level, p-level) data
  bool general = false;
  std::vector<pmg::dvec> verts;                  // per h-level
  std::vector<pmg::dvec> coef;                   // [hl * L + pl], empty = mu 1
  std::vector<pmg::QTabDev<double>> qt64;        // per p-level
  std::vector<pmg::QTabDev<float>> qt32;
  std::vector<const double *> G64, invD64;  // [hl * L + pl]
  std::vector<const float *> G32, invD32;
  std::vector<const pmg::bf16 *> G16, invD16;
  double *Ainv = nullptr, *cwork = nullptr; // dense coarse inverse and its gather vector
  int coarse_mi = 0;

  int nplev() const { return (int)degrees.size(); }
  long cells(int l) const { return dim == 3 ? (long)sizes[l] * sizes[l] * sizes[l] : (long)sizes[l] * sizes[l]; }
  long nodes(int l) const {
    long m = (long)p * sizes[l] + 1;
    return dim == 3 ? m * m * m : m * m;
  }
  int finest() const { return (int)sizes.size() - 1; }
  double cscale(int l) const { return dim == 3 ? 1.0 / sizes[l] : 1.0; }
  template <typename T>
  pmg::PrecData<T> &pd() {
    if constexpr (std::is_same<T, double>::value)
      return d64;
    else
      return d32;
  }
};

