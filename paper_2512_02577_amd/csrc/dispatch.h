// Compile-time dispatch over the supported degrees and p-hierarchies.
//
// Hierarchy code 0 is the paper's rule (Sec. 2.2: 1, 3, 7, ... below p, then p); code 1
// is the one-step hierarchy 1, 2, ..., p (offered for p <= 4).
#pragma once

#include "bodies.h"
#include "constants.h"

namespace pmg {

constexpr int kMaxDegree = 8;

// Calls F<P, Degrees<...>>::run(args...) for the runtime (p, code); returns -2 when the
// combination is not compiled in.
template <template <int, class> class F, typename... Args>
int dispatch_hierarchy(int p, int code, Args &&...args) {
  switch (code * 16 + p) {
    case 1: return F<1, Degrees<1>>::run(args...);
    case 2: return F<2, Degrees<1, 2>>::run(args...);
    case 3: return F<3, Degrees<1, 3>>::run(args...);
    case 4: return F<4, Degrees<1, 3, 4>>::run(args...);
    case 5: return F<5, Degrees<1, 3, 5>>::run(args...);
    case 6: return F<6, Degrees<1, 3, 6>>::run(args...);
    case 7: return F<7, Degrees<1, 3, 7>>::run(args...);
    case 8: return F<8, Degrees<1, 3, 7, 8>>::run(args...);
    case 16 + 1: return F<1, Degrees<1>>::run(args...);
    case 16 + 2: return F<2, Degrees<1, 2>>::run(args...);
    case 16 + 3: return F<3, Degrees<1, 2, 3>>::run(args...);
    case 16 + 4: return F<4, Degrees<1, 2, 3, 4>>::run(args...);
    default: return -2;
  }
}

// Calls F<P>::run(args...) for p = 1..8.
template <template <int> class F, typename... Args>
int dispatch_degree(int p, Args &&...args) {
  switch (p) {
    case 1: return F<1>::run(args...);
    case 2: return F<2>::run(args...);
    case 3: return F<3>::run(args...);
    case 4: return F<4>::run(args...);
    case 5: return F<5>::run(args...);
    case 6: return F<6>::run(args...);
    case 7: return F<7>::run(args...);
    case 8: return F<8>::run(args...);
    default: return -2;
  }
}

// Hierarchy code of a degree list (ascending), or -1 if not supported.
inline int hierarchy_code(int p, const int *deg, int L) {
  // paper rule
  {
    int q[8], k = 0, x = 1;
    while (x < p) { q[k++] = x; x = 2 * x + 1; }
    q[k++] = p;
    if (k == L) {
      bool same = true;
      for (int i = 0; i < L; ++i) same = same && q[i] == deg[i];
      if (same) return 0;
    }
  }
  if (p <= 4 && L == p) {
    bool same = true;
    for (int i = 0; i < L; ++i) same = same && deg[i] == i + 1;
    if (same) return 1;
  }
  return -1;
}

// Threads per workgroup of the patch kernel and of the apply kernel, by degree.  Up to degree
// 3 one wave per patch (its stages have at most 49 pencils); 3D patches that fit at most two
// per CU in LDS (degree 8, and degree 7 in FP64) get 8 waves, over which the contraction
// stages split their outputs.
constexpr int patch_threads(int p, int dim = 3, int tbytes = 8) {
  return p <= 3 ? 64 : (p <= 4 ? 128 : (p <= 6 || dim == 2 || (p == 7 && tbytes < 8) ? 256 : 512));
}
constexpr int apply_threads(int p) { return p <= 2 ? 128 : 128; }

// Lanes per patch and per cell of the general (metric) path: FP64 patches of degree >= 5
// fit one per CU in LDS, so they get 8 waves (the short stages split their outputs over
// them).
constexpr int metric_patch_threads(int p, int tbytes) { return p <= 2 ? 128 : (tbytes == 8 && p >= 5 ? 512 : 256); }
constexpr int metric_apply_threads(int p) { return p <= 3 ? 128 : 256; }


}  // namespace pmg
