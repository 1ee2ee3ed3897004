// Kernel bodies of the h-transfers between mesh levels and of the exact coarse solve
// (Sec. 2), written like the patch bodies: __host__ __device__, one output or one workgroup
// per call, so that a CPU build can run them for index and bounds checks.
#pragma once

#include "sumfac.h"

namespace pmg {

// ---------------------------------------------------------------------------------------
// h-transfers between mesh levels (Sec. 2): prolongation = embedding, restriction = its
// transpose.  With the Dirichlet rows and columns removed both are Kronecker products of
// one masked 1D matrix per direction, so each is applied as DIM passes of a 1D transfer,
// one thread per output entry.  1D weights: W1[alpha][a] = coarse cell basis a at the fine
// node alpha of the two fine cells inside the coarse cell; Wr[class][t] = restriction
// weights of a coarse node of class a = K mod P over its fine support (2P-1 nodes, 4P-1
// for a vertex).
// ---------------------------------------------------------------------------------------
template <typename T>
struct TransferArgs {
  const T *W1, *Wr;
  int nc;           // coarse cells per direction
  const T *in;
  T *out;
  T *w1, *w2;       // intermediates: >= mf*mf*mc and >= mf*mc*mc entries
  // restriction only, or nullptr: a coarse vector set to zero with the last pass (the zero
  // initial guess of the coarse correction; the restricted residual is zero on the boundary)
  T *zero;
};

template <typename T>
struct PassArgs {
  const T *W1, *Wr;
  int nc;
  int ax;           // contracted axis
  int ie[3], oe[3]; // input and output extents (x, y, z); 1 for unused axes
  const T *in;
  T *out;
  T *zero;          // nullptr, or set to zero at every output entry
};

template <typename T, int P, bool RESTRICT, bool ADD>
struct TransferPass {
  // output entry g of one pass
  PMG_INLINE static void node(long g, const PassArgs<T> &a) {
    const int o0 = (int)(g % a.oe[0]);
    const long r1 = g / a.oe[0];
    const int o1 = (int)(r1 % a.oe[1]);
    const int o2 = (int)(r1 / a.oe[1]);
    const int o[3] = {o0, o1, o2};
    const int istr[3] = {1, a.ie[0], a.ie[0] * a.ie[1]};
    const int ax = a.ax;
    long base = 0;
    for (int d = 0; d < 3; ++d)
      if (d != ax) base += (long)o[d] * istr[d];
    const long st = istr[ax];
    const cptr<T> W1 = as_const(a.W1), Wr = as_const(a.Wr);
    const int K = o[ax];
    // every tap is loaded (a fixed, unrolled count, the address clamped into range and the
    // weight of a missing tap zero), so that the loads of one output are in flight together
    T acc = 0;
    if (RESTRICT) {
      const int mc = P * a.nc + 1;
      const bool inner = K > 0 && K < mc - 1;  // coarse boundary rows vanish
      const int cc = K / P, cl = K % P;
      const int cnt = cl != 0 ? 2 * P - 1 : 4 * P - 1;
      int first = cl != 0 ? 2 * P * cc + 1 : 2 * P * (cc - 1) + 1;
      first = inner ? first : 1;
      constexpr int nw = 4 * P - 1;
      T x[nw];
#pragma unroll
      for (int t = 0; t < nw; ++t) {
        const T v = a.in[base + (long)(t < cnt ? first + t : first) * st];
        x[t] = t < cnt ? v : T(0);
      }
#pragma unroll
      for (int t = 0; t < nw; ++t) acc += Wr[cl * nw + t] * x[t];
      acc = inner ? acc : T(0);
    } else {
      const int mf = 2 * P * a.nc + 1, mc = P * a.nc + 1;
      const bool inner = K > 0 && K < mf - 1;  // fine boundary rows vanish
      int cc = K / (2 * P);
      if (cc > a.nc - 1) cc = a.nc - 1;
      const int al = K - 2 * P * cc;
      T x[P + 1];
#pragma unroll
      for (int c = 0; c <= P; ++c) {
        const int Kc = P * cc + c;
        const T v = a.in[base + (long)Kc * st];
        x[c] = Kc > 0 && Kc < mc - 1 ? v : T(0);
      }
#pragma unroll
      for (int c = 0; c <= P; ++c) acc += W1[al * (P + 1) + c] * x[c];
      acc = inner ? acc : T(0);
    }
    if (ADD)
      a.out[g] += acc;
    else
      a.out[g] = acc;
    if (a.zero) a.zero[g] = T(0);
  }
};

// Pass schedule of a transfer: restriction contracts x, y, z (fine -> coarse extent);
// prolongation expands x, y, z and adds the last pass into the fine vector.
template <typename T>
PMG_INLINE int transfer_passes(int dim, int P, bool restrict_, const TransferArgs<T> &t, PassArgs<T> pa[3]) {
  const int mc = P * t.nc + 1, mf = 2 * P * t.nc + 1;
  int cur[3] = {restrict_ ? mf : mc, restrict_ ? mf : mc, dim == 3 ? (restrict_ ? mf : mc) : 1};
  const int target = restrict_ ? mc : mf;
  const T *src = t.in;
  for (int ax = 0; ax < dim; ++ax) {
    PassArgs<T> &p = pa[ax];
    p.W1 = t.W1;
    p.Wr = t.Wr;
    p.nc = t.nc;
    p.ax = ax;
    for (int d = 0; d < 3; ++d) p.ie[d] = cur[d];
    cur[ax] = target;
    for (int d = 0; d < 3; ++d) p.oe[d] = cur[d];
    p.in = src;
    p.out = ax == dim - 1 ? t.out : (ax % 2 == 0 ? t.w1 : t.w2);
    p.zero = restrict_ && ax == dim - 1 ? t.zero : nullptr;
    src = p.out;
  }
  return dim;
}

// ---------------------------------------------------------------------------------------
// Coarsest mesh: z = A_0^{-1} r by fast diagonalization of the Cartesian interior operator,
// A_0 = c0 sum_k K (x) M (x) M with K S = M S diag(lam), S^T M S = I, so
// A_0^{-1} = (1/c0) (S (x) S (x) S) diag(1 / (lam_i + lam_j + lam_k)) (S (x) S (x) S)^T.
// One workgroup; w1/w2 are float64 work arrays of m^d entries.  Boundary: z = r.
// ---------------------------------------------------------------------------------------
template <typename T>
struct CoarseArgs {
  const double *S, *lam;
  double c0inv;
  int m;   // interior nodes per direction
  int mt;  // total nodes per direction (m + 2)
  const T *r;
  T *z;
  double *w1, *w2;
};

template <int DIM, typename T, int NT>
struct CoarseBody {
  // w_out(.., a, ..) = sum_i S[i][a] w_in(.., i, ..) (transpose) or sum_a S[i][a] w_in(..a..)
  PMG_INLINE static void axis(int tid, const CoarseArgs<T> &a, const double *in, double *out, int ax, bool tr) {
    const int m = a.m, tot = DIM == 3 ? m * m * m : m * m;
    const int st = ax == 0 ? 1 : (ax == 1 ? m : m * m);
    for (int e = tid; e < tot; e += NT) {
      const int o = (e / st) % m, base = e - o * st;
      double s = 0.0;
#pragma unroll 4
      for (int i = 0; i < m; ++i) s += (tr ? a.S[i * m + o] : a.S[o * m + i]) * in[base + i * st];
      out[e] = s;
    }
  }
  // lds: lds_elems doubles of workgroup memory; when both work vectors fit there the passes
  // run on it instead of on the global buffers w1, w2
  PMG_INLINE static void run(int tid, const CoarseArgs<T> &a, double *lds = nullptr, int lds_elems = 0) {
    const int m = a.m, mt = a.mt, tot = DIM == 3 ? m * m * m : m * m;
    const bool inl = lds != nullptr && 2 * tot <= lds_elems;
    double *const w1 = inl ? lds : a.w1, *const w2 = inl ? lds + tot : a.w2;
    const int totall = DIM == 3 ? mt * mt * mt : mt * mt;
    for (int e = tid; e < totall; e += NT) {  // boundary rows are identity rows
      const int i = e % mt, j = (e / mt) % mt, k = DIM == 3 ? e / (mt * mt) : 1;
      bool bnd = i == 0 || i == mt - 1 || j == 0 || j == mt - 1;
      if (DIM == 3) bnd = bnd || k == 0 || k == mt - 1;
      if (bnd) a.z[e] = a.r[e];
    }
    for (int e = tid; e < tot; e += NT) {
      const int i = e % m, j = (e / m) % m, k = DIM == 3 ? e / (m * m) : 0;
      w1[e] = (double)a.r[(i + 1) + mt * ((j + 1) + mt * (k + (DIM == 3 ? 1 : 0)))];
    }
    PMG_SYNC();
    double *x = w1, *y = w2;
    for (int ax = 0; ax < DIM; ++ax) {
      axis(tid, a, x, y, ax, true);
      PMG_SYNC();
      double *t = x; x = y; y = t;
    }
    for (int e = tid; e < tot; e += NT) {
      const int i = e % m, j = (e / m) % m, k = DIM == 3 ? e / (m * m) : 0;
      double lsum = a.lam[i] + a.lam[j] + (DIM == 3 ? a.lam[k] : 0.0);
      x[e] *= a.c0inv / lsum;
    }
    PMG_SYNC();
    for (int ax = 0; ax < DIM; ++ax) {
      axis(tid, a, x, y, ax, false);
      PMG_SYNC();
      double *t = x; x = y; y = t;
    }
    for (int e = tid; e < tot; e += NT) {
      const int i = e % m, j = (e / m) % m, k = DIM == 3 ? e / (m * m) : 0;
      a.z[(i + 1) + mt * ((j + 1) + mt * (k + (DIM == 3 ? 1 : 0)))] = (T)x[e];
    }
  }
};

}  // namespace pmg
