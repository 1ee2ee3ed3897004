// Runtime dispatch from (dimension, precision) to the instantiated launchers.
#include "launch.h"

namespace pmg {

size_t patch_arena_bytes(int dim, int prec, int p, int hcode) {
  if (prec == 0) return dim == 3 ? Launchers<3, double>::patch_bytes(p, hcode) : Launchers<2, double>::patch_bytes(p, hcode);
  return dim == 3 ? Launchers<3, float>::patch_bytes(p, hcode) : Launchers<2, float>::patch_bytes(p, hcode);
}

size_t apply_arena_bytes(int dim, int prec, int p) {
  if (prec == 0) return dim == 3 ? Launchers<3, double>::apply_bytes(p) : Launchers<2, double>::apply_bytes(p);
  return dim == 3 ? Launchers<3, float>::apply_bytes(p) : Launchers<2, float>::apply_bytes(p);
}

size_t metric_patch_arena_bytes(int dim, int prec, int p) {
  if (prec == 0) return dim == 3 ? MetricLaunchers<3, double, double>::patch_bytes(p) : MetricLaunchers<2, double, double>::patch_bytes(p);
  return dim == 3 ? MetricLaunchers<3, float, float>::patch_bytes(p) : MetricLaunchers<2, float, float>::patch_bytes(p);
}

size_t metric_apply_arena_bytes(int dim, int prec, int p) {
  if (prec == 0) return dim == 3 ? MetricLaunchers<3, double, double>::apply_bytes(p) : MetricLaunchers<2, double, double>::apply_bytes(p);
  return dim == 3 ? MetricLaunchers<3, float, float>::apply_bytes(p) : MetricLaunchers<2, float, float>::apply_bytes(p);
}

template <typename T>
int launch_smooth_color(int dim, int p, int hcode, const SmoothArgs<T> &a, const Arena &ar, hipStream_t s) {
  return dim == 3 ? Launchers<3, T>::smooth(p, hcode, a, ar, s) : Launchers<2, T>::smooth(p, hcode, a, ar, s);
}

template <typename T>
int launch_local_only(int dim, int p, int hcode, const SmoothArgs<T> &a, int n_blocks, const Arena &ar,
                      hipStream_t s) {
  return dim == 3 ? Launchers<3, T>::local(p, hcode, a, n_blocks, ar, s)
                  : Launchers<2, T>::local(p, hcode, a, n_blocks, ar, s);
}

template <typename T>
int launch_apply(int dim, int p, int kind, const ApplyArgs<T> &a, const Arena &ar, hipStream_t s) {
  return dim == 3 ? Launchers<3, T>::apply(p, kind, a, ar, s) : Launchers<2, T>::apply(p, kind, a, ar, s);
}

template <typename T>
int launch_restrict(int dim, int p, const TransferArgs<T> &a, hipStream_t s) {
  return dim == 3 ? Launchers<3, T>::restrict_(p, a, s) : Launchers<2, T>::restrict_(p, a, s);
}

template <typename T>
int launch_prolong_add(int dim, int p, const TransferArgs<T> &a, hipStream_t s) {
  return dim == 3 ? Launchers<3, T>::prolong(p, a, s) : Launchers<2, T>::prolong(p, a, s);
}

template <typename T>
int launch_coarse(int dim, const CoarseArgs<T> &a, hipStream_t s) {
  return dim == 3 ? Launchers<3, T>::coarse(a, s) : Launchers<2, T>::coarse(a, s);
}

#define PMG_INSTANTIATE(T)                                                                              \
  template int launch_smooth_color<T>(int, int, int, const SmoothArgs<T> &, const Arena &, hipStream_t); \
  template int launch_local_only<T>(int, int, int, const SmoothArgs<T> &, int, const Arena &, hipStream_t); \
  template int launch_apply<T>(int, int, int, const ApplyArgs<T> &, const Arena &, hipStream_t);       \
  template int launch_restrict<T>(int, int, const TransferArgs<T> &, hipStream_t);                       \
  template int launch_prolong_add<T>(int, int, const TransferArgs<T> &, hipStream_t);                    \
  template int launch_coarse<T>(int, const CoarseArgs<T> &, hipStream_t);

PMG_INSTANTIATE(double)
PMG_INSTANTIATE(float)

}  // namespace pmg
