// Kernel bodies of the general path: distorted cells and a variable coefficient.
//
// The operator is evaluated by sum factorization through the Gauss points (Sec. 3,
// "evaluation kernel" with the coefficient mu at quadrature points, Sec. 4 distorted
// meshes): nodal values -> values at Gauss points (B in each direction) -> reference
// gradient (collocation derivative Dq in each direction) -> flux G grad (G the stored
// symmetric metric w mu |det J| J^-1 J^-T) -> transposed derivative and basis sweeps.
// On a patch the two cells per direction form one tensor of 2(q+1) Gauss points; the 1D
// patch matrices are block-structured (each Gauss point sees the nodes of its own cell).
//
// G is stored per cell and Gauss point in the storage type S (double, float or bfloat16
// bits), components (xx, yy, zz, xy, xz, yz) in 3D and (xx, yy, xy) in 2D.
#pragma once

#include <type_traits>

#include "bodies.h"

namespace pmg {

// ---- storage type conversion (bfloat16 kept as raw 16-bit patterns) ----
struct bf16 {
  unsigned short bits;
};

template <typename T, typename S>
PMG_INLINE T load_s(const S *p, long i) {
  return (T)p[i];
}
template <>
PMG_INLINE float load_s<float, bf16>(const bf16 *p, long i) {
  const unsigned int u = ((unsigned int)p[i].bits) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
template <>
PMG_INLINE double load_s<double, bf16>(const bf16 *p, long i) {
  return (double)load_s<float, bf16>(p, i);
}

template <typename S>
PMG_INLINE S to_storage(double v) {
  return (S)v;
}
template <>
PMG_INLINE bf16 to_storage<bf16>(double v) {  // round to nearest even
  const float f = (float)v;
  unsigned int u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  bf16 r;
  r.bits = (unsigned short)(u >> 16);
  return r;
}

// ---- sparsity patterns of the patch Gauss-point matrices (degree Q, NQ = Q+1 per cell) ----
template <int Q>
struct PatBpc {  // 2NQ x (2Q+1): closure nodes -> patch Gauss points
  static constexpr int nq = Q + 1, nout = 2 * nq, nin = 2 * Q + 1;
  PMG_HD static constexpr int lo(int r) { return (r / nq) * Q; }
  PMG_HD static constexpr int hi(int r) { return (r / nq) * Q + Q + 1; }
};
template <int Q>
struct PatBpi {  // 2NQ x (2Q-1): interior nodes -> patch Gauss points
  static constexpr int nq = Q + 1, nout = 2 * nq, nin = 2 * Q - 1;
  PMG_HD static constexpr int lo(int r) { return r / nq ? Q - 1 : 0; }
  PMG_HD static constexpr int hi(int r) { return r / nq ? 2 * Q - 1 : Q; }
};
template <int Q>
struct PatBpiT {  // (2Q-1) x 2NQ
  static constexpr int nq = Q + 1, nout = 2 * Q - 1, nin = 2 * nq;
  PMG_HD static constexpr int lo(int c) { return c + 1 > Q ? nq : 0; }
  PMG_HD static constexpr int hi(int c) { return c + 1 < Q ? nq : 2 * nq; }
};
template <int Q>
struct PatDqp {  // 2NQ x 2NQ block diagonal (also its transpose)
  static constexpr int nq = Q + 1, nout = 2 * nq, nin = 2 * nq;
  PMG_HD static constexpr int lo(int r) { return (r / nq) * nq; }
  PMG_HD static constexpr int hi(int r) { return (r / nq) * nq + nq; }
};
// out = base - Mat in  along an axis (base may alias out)
template <int AX, int E0, int E1, int E2, class Pat, int NT, typename T>
PMG_INLINE void contract_sub(int tid, const T *in, T *out, const T *base, const T *Mat_) {
  using X = Axis<AX, E0, E1, E2, Pat::nout>;
  static_assert(X::NIN == Pat::nin, "extent mismatch");
  const cptr<T> Mat0 = as_const(Mat_);
  for (int pen = tid; pen < X::NPEN; pen += NT) {
    const cptr<T> Mat = per_pencil(Mat0);
    int ib, obs;
    X::base(pen, ib, obs);
    T v[Pat::nin];
#pragma unroll
    for (int i = 0; i < Pat::nin; ++i) v[i] = in[ib + i * X::IS];
#pragma unroll
    for (int o = 0; o < Pat::nout; ++o) {
      const T acc = row1<Pat>(Mat, o, v);
      const int oi = obs + o * X::OS;
      out[oi] = base[oi] - acc;
    }
  }
}

// Global index of the cell at block position (dx, dy, dz) of a patch (or of one cell).
struct BoxCells {  // structured n^d box, the block starting at cell c0
  int n, c0[3];
  PMG_HD long operator()(int dx, int dy, int dz) const {
    return (long)(c0[0] + dx) + (long)n * ((c0[1] + dy) + (long)n * (c0[2] + dz));
  }
};
struct ListCells {  // stored per patch: its cells in block order dx + 2 dy + 4 dz
  const int32_t *id;
  PMG_HD long operator()(int dx, int dy, int dz) const { return id[dx + 2 * dy + 4 * dz]; }
};
struct OneCell {
  long c;
  PMG_HD long operator()(int, int, int) const { return c; }
};

// Pointwise flux F = G g on NQ^DIM Gauss points held in gx/gy/gz (overwritten).  The
// metric of point (i, j, k) lives in cell cm(i / nq, ...) at local point (i % nq, ...).
template <int DIM, int NQ, int nq, int NT, typename T, typename S, class CM>
PMG_INLINE void flux(int tid, T *gx, T *gy, T *gz, const S *G, const CM &cm) {
  constexpr int tot = ipow(NQ, DIM), nqd = ipow(nq, DIM), nc = DIM == 3 ? 6 : 3;
  // the metric loads of GF points per lane are issued together (one round trip per group)
  constexpr int RF = (tot + NT - 1) / NT, GF = RF < 3 ? RF : 3;
  for (int k0 = 0; k0 < RF; k0 += GF) {
    T g[GF][nc];
#pragma unroll
    for (int k = 0; k < GF; ++k) {
      int e = tid + (k0 + k) * NT;
      e = e < tot ? e : tot - 1;
      const int i = e % NQ, j = (e / NQ) % NQ, l = DIM == 3 ? e / (NQ * NQ) : 0;
      const long cell = cm(i / nq, j / nq, DIM == 3 ? l / nq : 0);
      const int loc = (i % nq) + nq * ((j % nq) + nq * (DIM == 3 ? l % nq : 0));
      const long gi = (cell * nqd + loc) * nc;
#pragma unroll
      for (int c = 0; c < nc; ++c) g[k][c] = load_s<T>(G, gi + c);
    }
#pragma unroll
    for (int k = 0; k < GF; ++k) {
      const int e = tid + (k0 + k) * NT;
      if (k0 + k >= RF || e >= tot) continue;
      const T a = gx[e], b = gy[e];
      if (DIM == 3) {
        const T c = gz[e];
        const T xx = g[k][0], yy = g[k][1], zz = g[k][2], xy = g[k][3], xz = g[k][4], yz = g[k][5];
        gx[e] = xx * a + xy * b + xz * c;
        gy[e] = xy * a + yy * b + yz * c;
        gz[e] = xz * a + yz * b + zz * c;
      } else {
        const T xx = g[k][0], yy = g[k][1], xy = g[k][2];
        gx[e] = xx * a + xy * b;
        gy[e] = xy * a + yy * b;
      }
    }
  }
}

// 1D tables of one degree for the metric path (device pointers)
template <typename T>
struct QTabDev {
  const T *B, *BT, *Dq, *DqT, *Bpc, *Bpi, *BpiT, *Dqp, *DqpT;
};

// Scratch of metric_patch on a patch of degree Q: three (2D: two) buffers A, B, C of NQ^d
// Gauss-point values.  The interpolation stages to the Gauss points run through B and C,
// the values land in A; the y and z reference derivatives go to B and C, the x derivative
// replaces the values in A (in place along x); the flux is formed in place; the
// transposed derivatives accumulate in A (x in place first); the stages back to the nodes
// run through B and C.
template <int DIM, int Q>
struct MetricScratch {
  static constexpr int NQ = 2 * (Q + 1);
  static constexpr int q3 = ipow(NQ, DIM);
  static constexpr int total = (DIM == 3 ? 3 : 2) * q3;
};

// out = base - A_patch in, with A evaluated through the Gauss points of the patch's cells.
// PB: pattern of the input sweep (PatBpc for closure input, PatBpi for interior input).
template <int DIM, int Q, class PB, int NT, typename T, typename S, class CM>
PMG_INLINE void metric_patch(int tid, const T *in, T *out, const T *base, const QTabDev<T> &tb, const S *G,
                             const CM &cm, T *scr) {
  constexpr int E = PB::nin, NQ = 2 * (Q + 1), nq = Q + 1, e = 2 * Q - 1;
  using SC = MetricScratch<DIM, Q>;
  using PD = PatDqp<Q>;
  using PT = PatBpiT<Q>;
  T *A = scr, *B = scr + SC::q3, *C = DIM == 3 ? scr + 2 * SC::q3 : nullptr;
  static_assert(DIM == 2 || (NQ * E * E <= SC::q3 && NQ * NQ * E <= SC::q3 && e * NQ * NQ <= SC::q3),
                "interpolation stages must fit a Gauss-point buffer");
  const T *Bin = std::is_same<PB, PatBpc<Q>>::value ? tb.Bpc : tb.Bpi;
  if constexpr (DIM == 3) {
    dcontract1<0, E, E, E, PB, NT, false>(tid, in, B, Bin);
    PMG_SYNC();
    dcontract1<1, NQ, E, E, PB, NT, false>(tid, B, C, Bin);
    PMG_SYNC();
    dcontract1<2, NQ, NQ, E, PB, NT, false>(tid, C, A, Bin);  // values at the Gauss points
    PMG_SYNC();
    dcontract1<1, NQ, NQ, NQ, PD, NT, false>(tid, A, B, tb.Dqp);
    dcontract1<2, NQ, NQ, NQ, PD, NT, false>(tid, A, C, tb.Dqp);
    PMG_SYNC();
    dcontract1<0, NQ, NQ, NQ, PD, NT, false, true>(tid, A, A, tb.Dqp);
    PMG_SYNC();
    flux<3, NQ, nq, NT>(tid, A, B, C, G, cm);
    PMG_SYNC();
    dcontract1<0, NQ, NQ, NQ, PD, NT, false, true>(tid, A, A, tb.DqpT);
    PMG_SYNC();
    dcontract1<1, NQ, NQ, NQ, PD, NT, true>(tid, B, A, tb.DqpT);
    PMG_SYNC();
    dcontract1<2, NQ, NQ, NQ, PD, NT, true>(tid, C, A, tb.DqpT);
    PMG_SYNC();
    dcontract1<0, NQ, NQ, NQ, PT, NT, false>(tid, A, B, tb.BpiT);
    PMG_SYNC();
    dcontract1<1, e, NQ, NQ, PT, NT, false>(tid, B, C, tb.BpiT);
    PMG_SYNC();
    dcontract_sub<2, e, e, NQ, PT, NT>(tid, C, out, base, tb.BpiT);
  } else {
    dcontract1<0, E, E, 1, PB, NT, false>(tid, in, B, Bin);
    PMG_SYNC();
    dcontract1<1, NQ, E, 1, PB, NT, false>(tid, B, A, Bin);
    PMG_SYNC();
    dcontract1<1, NQ, NQ, 1, PD, NT, false>(tid, A, B, tb.Dqp);
    PMG_SYNC();
    dcontract1<0, NQ, NQ, 1, PD, NT, false, true>(tid, A, A, tb.Dqp);
    PMG_SYNC();
    flux<2, NQ, nq, NT>(tid, A, B, B, G, cm);
    PMG_SYNC();
    dcontract1<0, NQ, NQ, 1, PD, NT, false, true>(tid, A, A, tb.DqpT);
    PMG_SYNC();
    dcontract1<1, NQ, NQ, 1, PD, NT, true>(tid, B, A, tb.DqpT);
    PMG_SYNC();
    dcontract1<0, NQ, NQ, 1, PT, NT, false>(tid, A, B, tb.BpiT);
    PMG_SYNC();
    dcontract_sub<1, e, NQ, 1, PT, NT>(tid, B, out, base, tb.BpiT);
  }
}

// ---------------------------------------------------------------------------------------
// Patch smoother of the general path (Alg. 1 body, Alg. 2, Alg. 3 with the metric vmult
// and per-patch inverse diagonals).
// ---------------------------------------------------------------------------------------
template <typename T, typename S>
struct MetricLevelDev {
  QTabDev<T> qt;
  const T *Tp, *TpT;  // embedding from the next coarser p-level (level > 0)
  const S *G;         // metric of this h-level at this degree
  const S *invD;      // per patch, (2q-1)^d entries each, damping folded in
};

template <typename T, typename S>
struct MetricSmoothArgs {
  MetricLevelDev<T, S> lev[4];
  int n;
  int first[3], cnt[3], n_patch;
  int full, n_iter;
  T *u;
  const T *b;
  const T *r_blocks;
  T *d_blocks;
  int first_patch;
  // stored maps of a general hex mesh (null on the structured box): the patches of the
  // color, each patch's (2p+1)^d closure nodes (-1 on the boundary) and its 2^d cells
  const int32_t *plist, *pmap, *pcells;
};

template <int DIM, typename T, typename S, int NT, int P, class H>
struct MetricPatchBody {
  static constexpr int L = H::L;
  static_assert(H::q[L - 1] == P && H::q[0] == 1, "hierarchy must run from 1 to the degree");
  static constexpr int N = 2 * P + 1, n = 2 * P - 1;
  static constexpr int Nd = ipow(N, DIM), nd = ipow(n, DIM);
  static constexpr int qd(int l) { return H::q[l]; }
  static constexpr int nl(int l) { return 2 * H::q[l] - 1; }
  static constexpr int ndl(int l) { return ipow(2 * H::q[l] - 1, DIM); }
  static constexpr int scratch(int l) {  // MetricScratch<DIM, q_l>::total
    return (DIM == 3 ? 3 : 2) * ipow(2 * (qd(l) + 1), DIM);
  }
  static constexpr int transfer_scratch(int l) {
    return l == 0 ? 0
                  : cmax(kron_t1(DIM, nl(l), nl(l - 1)) + kron_t2(DIM, nl(l), nl(l - 1)),
                         kron_t1(DIM, nl(l - 1), nl(l)) + kron_t2(DIM, nl(l - 1), nl(l)));
  }
  static constexpr int scr_size() {
    int s = scratch(L - 1);
    for (int l = 1; l < L; ++l) s = cmax(s, cmax(scratch(l), transfer_scratch(l)));
    return s;
  }
  // layout: r | d | lower r_l, d_l | res | scratch | c (Richardson steps after the first
  // only, so that one step needs `size1`).  The closure values ucl (phase R only) overlay
  // lower, res and the start of the scratch: the first interpolation stage reads ucl and
  // writes the second scratch buffer, beyond ucl.
  static constexpr int off_r = 0, off_d = nd, off_ucl = 2 * nd;
  static constexpr int lower_size(int l) { return l < 0 ? 0 : 2 * ndl(l) + lower_size(l - 1); }
  static constexpr int off_lr(int l) { return 2 * nd + (l == 0 ? 0 : lower_size(l - 1)); }
  static constexpr int off_ld(int l) { return off_lr(l) + ndl(l); }
  static constexpr int off_res = 2 * nd + lower_size(L - 2);
  static constexpr int off_scr = off_res + nd;
  static_assert(off_ucl + Nd <= off_scr + ipow(2 * (P + 1), DIM), "closure must end before the stage-1 buffer");
  static constexpr int size1 = off_scr + scr_size();
  static constexpr int off_cc = size1;
  static constexpr int size = size1 + nd;
  PMG_HD static constexpr int arena(int n_iter) { return n_iter > 1 ? size : size1; }

  // out (=|+=) Kronecker product of Mat in every direction, on compact tensors
  template <class Pat, bool ADD>
  PMG_INLINE static void kron_dense(int tid, const T *in, T *out, const T *Mat, T *t1, T *t2) {
    constexpr int I = Pat::nin, O = Pat::nout;
    if constexpr (DIM == 3) {
      dcontract1<0, I, I, I, Pat, NT, false>(tid, in, t1, Mat);
      PMG_SYNC();
      dcontract1<1, O, I, I, Pat, NT, false>(tid, t1, t2, Mat);
      PMG_SYNC();
      dcontract1<2, O, O, I, Pat, NT, ADD>(tid, t2, out, Mat);
    } else {
      dcontract1<0, I, I, 1, Pat, NT, false>(tid, in, t1, Mat);
      PMG_SYNC();
      dcontract1<1, O, I, 1, Pat, NT, ADD>(tid, t1, out, Mat);
    }
  }

  template <int l, class CM>
  PMG_INLINE static void vmult_residual(int tid, T *lds, const MetricSmoothArgs<T, S> &a, const CM &cm,
                                        const T *d, const T *r, T *res) {
    metric_patch<DIM, qd(l), PatBpi<qd(l)>, NT>(tid, d, res, r, a.lev[l].qt, a.lev[l].G, cm, lds + off_scr);
  }

  template <int l, class CM>
  PMG_INLINE static void cycle(int tid, T *lds, const MetricSmoothArgs<T, S> &a, long pidx, const CM &cm,
                               const T *r, T *d, bool full) {
    const S *invD = a.lev[l].invD + pidx * ndl(l);
    if constexpr (l == 0) {
      if (tid == 0) d[0] = load_s<T>(invD, 0) * r[0];
      PMG_SYNC();
    } else {
      constexpr int q = qd(l), qc = qd(l - 1), ndq = ndl(l);
      constexpr int t1size = DIM == 3 ? cmax(kron_t1(DIM, nl(l), nl(l - 1)), kron_t1(DIM, nl(l - 1), nl(l))) : 0;
      lane_gather<ndq, NT, 16, T>(
          tid, [&](int e) { return load_s<T>(invD, e); }, [&](int e, T x) { d[e] = x * r[e]; });
      PMG_SYNC();
      T *res = lds + off_res;
      vmult_residual<l>(tid, lds, a, cm, d, r, res);
      PMG_SYNC();
      T *rc = lds + off_lr(l - 1), *dc = lds + off_ld(l - 1);
      T *t1 = lds + off_scr, *t2 = t1 + t1size;
      kron_dense<PatRestrict<q, qc>, false>(tid, res, rc, a.lev[l].TpT, t1, t2);
      PMG_SYNC();
      cycle<l - 1>(tid, lds, a, pidx, cm, rc, dc, full);
      kron_dense<PatProlong<q, qc>, true>(tid, dc, d, a.lev[l].Tp, t1, t2);
      PMG_SYNC();
      if (full) {
        vmult_residual<l>(tid, lds, a, cm, d, r, res);
        PMG_SYNC();
        lane_gather<ndq, NT, 16, T>(
            tid, [&](int e) { return load_s<T>(invD, e); }, [&](int e, T x) { d[e] += x * res[e]; });
        PMG_SYNC();
      }
    }
  }

  // ONE: the local solver is one half V-cycle (the default), compiled without the code of
  // the other variants
  template <bool ONE = false, class CM>
  PMG_INLINE static void local_solve(int tid, T *lds, const MetricSmoothArgs<T, S> &a, long pidx, const CM &cm) {
    T *r = lds + off_r, *d = lds + off_d, *cc = lds + off_cc;
    if constexpr (ONE) {
      cycle<L - 1>(tid, lds, a, pidx, cm, r, d, false);
      return;
    }
    const bool full = a.full != 0;
    cycle<L - 1>(tid, lds, a, pidx, cm, r, d, full);
    for (int it = 1; it < a.n_iter; ++it) {
      vmult_residual<L - 1>(tid, lds, a, cm, it == 1 ? d : cc, r, r);
      PMG_SYNC();
      cycle<L - 1>(tid, lds, a, pidx, cm, r, cc, full);
      for (int e = tid; e < nd; e += NT) d[e] += cc[e];
      PMG_SYNC();
    }
  }

  PMG_INLINE static void vertex(int pidx_color, const MetricSmoothArgs<T, S> &a, int v[3]) {
    v[0] = a.first[0] + 2 * (pidx_color % a.cnt[0]);
    v[1] = a.first[1] + 2 * ((pidx_color / a.cnt[0]) % a.cnt[1]);
    v[2] = DIM == 3 ? a.first[2] + 2 * (pidx_color / (a.cnt[0] * a.cnt[1])) : 0;
  }

  PMG_INLINE static long patch_index(const int v[3], int ncell) {
    return (long)(v[0] - 1) + (long)(ncell - 1) * ((v[1] - 1) + (long)(ncell - 1) * (DIM == 3 ? v[2] - 1 : 0));
  }

  template <bool ONE = false>
  PMG_INLINE static void smooth_patch(int tid, int blk, T *lds, const MetricSmoothArgs<T, S> &a) {
    int v[3];
    vertex(xcd_remap(blk, a.n_patch), a, v);
    const long pidx = patch_index(v, a.n);
    const int c0[3] = {v[0] - 1, v[1] - 1, DIM == 3 ? v[2] - 1 : 0};
    const int m = P * a.n + 1;
    const int g0[3] = {P * (v[0] - 1), P * (v[1] - 1), DIM == 3 ? P * (v[2] - 1) : 0};
    T *ucl = lds + off_ucl, *r = lds + off_r;
    const int ez = DIM == 3 ? 1 : 0;
    auto interior = [&](int e) {
      const int i = e % n, j = (e / n) % n, k = DIM == 3 ? e / (n * n) : 0;
      return (g0[0] + 1 + i) + (long)m * ((g0[1] + 1 + j) + (long)m * (g0[2] + ez + k));
    };
    // closure of u (zero on the Dirichlet boundary; every closure node lies inside the
    // mesh, so the load itself is always valid) and the interior of b, loads batched
    lane_gather2<Nd, nd, NT, 16, T>(
        tid,
        [&](int e) {
          const int i = e % N, j = (e / N) % N, k = DIM == 3 ? e / (N * N) : 0;
          const int gx = g0[0] + i, gy = g0[1] + j, gz = g0[2] + k;
          bool bnd = gx == 0 || gx == m - 1 || gy == 0 || gy == m - 1;
          if (DIM == 3) bnd = bnd || gz == 0 || gz == m - 1;
          const T x = a.u[gx + (long)m * (gy + (long)m * gz)];
          return bnd ? T(0) : x;
        },
        [&](int e, T x) { ucl[e] = x; }, [&](int e) { return a.b[interior(e)]; }, [&](int e, T x) { r[e] = x; });
    PMG_SYNC();
    const BoxCells cm{a.n, {c0[0], c0[1], c0[2]}};
    metric_patch<DIM, P, PatBpc<P>, NT>(tid, ucl, r, r, a.lev[L - 1].qt, a.lev[L - 1].G, cm, lds + off_scr);
    PMG_SYNC();
    local_solve<ONE>(tid, lds, a, pidx, cm);
    const T *d = lds + off_d;
    lane_gather<nd, NT, 16, T>(
        tid, [&](int e) { return a.u[interior(e)]; }, [&](int e, T x) { a.u[interior(e)] = x + d[e]; });
  }

  // The same on a general hex mesh through its stored maps: the color's patch list, the
  // patch's closure nodes (-1 on the Dirichlet boundary, gathered as zero) and its cells.
  template <bool ONE = false>
  PMG_INLINE static void smooth_patch_stored(int tid, int blk, T *lds, const MetricSmoothArgs<T, S> &a) {
    const long pidx = a.plist[xcd_remap(blk, a.n_patch)];
    const int32_t *cl = a.pmap + pidx * Nd;
    T *ucl = lds + off_ucl, *r = lds + off_r;
    const int ez = DIM == 3 ? 1 : 0;
    auto interior = [&](int e) {  // closure position of interior node e
      const int i = e % n, j = (e / n) % n, k = DIM == 3 ? e / (n * n) : 0;
      return (i + 1) + N * ((j + 1) + N * (k + ez));
    };
    lane_gather2<Nd, nd, NT, 16, T>(
        tid,
        [&](int e) {
          const int g = cl[e];
          return g >= 0 ? a.u[g] : T(0);
        },
        [&](int e, T x) { ucl[e] = x; }, [&](int e) { return a.b[cl[interior(e)]]; }, [&](int e, T x) { r[e] = x; });
    PMG_SYNC();
    const ListCells cm{a.pcells + pidx * (1 << DIM)};
    metric_patch<DIM, P, PatBpc<P>, NT>(tid, ucl, r, r, a.lev[L - 1].qt, a.lev[L - 1].G, cm, lds + off_scr);
    PMG_SYNC();
    local_solve<ONE>(tid, lds, a, pidx, cm);
    const T *d = lds + off_d;
    lane_gather<nd, NT, 16, T>(
        tid, [&](int e) { return a.u[cl[interior(e)]]; }, [&](int e, T x) { a.u[cl[interior(e)]] = x + d[e]; });
  }

  PMG_INLINE static void local_only(int tid, int blk, T *lds, const MetricSmoothArgs<T, S> &a) {
    const long pidx = a.first_patch + blk;
    const long k1 = a.n - 1;
    const int v[3] = {(int)(pidx % k1) + 1, (int)((pidx / k1) % k1) + 1, DIM == 3 ? (int)(pidx / (k1 * k1)) + 1 : 0};
    const int c0[3] = {v[0] - 1, v[1] - 1, DIM == 3 ? v[2] - 1 : 0};
    T *r = lds + off_r;
    const size_t base = (size_t)blk * nd;
    lane_gather<nd, NT, 16, T>(tid, [&](int e) { return a.r_blocks[base + e]; }, [&](int e, T x) { r[e] = x; });
    PMG_SYNC();
    local_solve(tid, lds, a, pidx, BoxCells{a.n, {c0[0], c0[1], c0[2]}});
    const T *d = lds + off_d;
    for (int e = tid; e < nd; e += NT) a.d_blocks[base + e] = d[e];
  }
};

// ---------------------------------------------------------------------------------------
// Cellwise apply of the general operator: cells of one parity color (they share no node)
// each add their element contribution into out (out = out + sign * A_K u_K); a separate
// init pass sets out = b (residual) or 0 (apply) on interior nodes and the Dirichlet
// identity rows.
// ---------------------------------------------------------------------------------------
template <typename T, typename S>
struct MetricApplyArgs {
  QTabDev<T> qt;
  const S *G;
  int n;          // cells per direction
  int first[3];   // first cell coordinate of the color per axis (0 or 1)
  int cnt[3];     // cells of the color per axis
  int n_cells;
  T sign;         // +1 apply, -1 residual
  const T *u;
  T *out;
  // stored maps of a general hex mesh (null on the structured box): the cells of the
  // color and each cell's (p+1)^d nodes; bnd marks the Dirichlet nodes
  const int32_t *clist, *cdof;
  const unsigned char *bnd;
};

template <int DIM, typename T, typename S, int NT, int P>
struct MetricApplyBody {
  static constexpr int k = P + 1, nq = P + 1;
  static constexpr int kd = ipow(k, DIM), q3 = ipow(nq, DIM);
  static constexpr int w1 = DIM == 3 ? nq * k * k : nq * k;
  static constexpr int w2 = DIM == 3 ? nq * nq * k : 0;
  static constexpr int size = kd + w1 + w2 + (DIM == 3 ? 4 : 3) * q3;

  // STORED: the cell and its nodes come from the stored maps of a general hex mesh
  template <bool STORED = false>
  PMG_INLINE static void run(int tid, int blk, T *lds, const MetricApplyArgs<T, S> &a) {
    const int idx = xcd_remap(blk, a.n_cells);
    int cx = 0, cy = 0, cz = 0;
    long cell = 0;
    if constexpr (STORED) {
      cell = a.clist[idx];
    } else {
      cx = a.first[0] + 2 * (idx % a.cnt[0]);
      cy = a.first[1] + 2 * ((idx / a.cnt[0]) % a.cnt[1]);
      cz = DIM == 3 ? a.first[2] + 2 * (idx / (a.cnt[0] * a.cnt[1])) : 0;
      cell = cx + (long)a.n * (cy + (long)a.n * cz);
    }
    const int m = P * a.n + 1;
    // global index of cell node e and whether it is a Dirichlet node
    auto node = [&](int e, bool &bnd) -> long {
      if constexpr (STORED) {
        const long g = a.cdof[cell * kd + e];
        bnd = a.bnd[g] != 0;
        return g;
      } else {
        const int i = e % k, j = (e / k) % k, l = DIM == 3 ? e / (k * k) : 0;
        const int X = P * cx + i, Y = P * cy + j, Z = P * cz + l;
        bnd = X == 0 || X == m - 1 || Y == 0 || Y == m - 1;
        if (DIM == 3) bnd = bnd || Z == 0 || Z == m - 1;
        return X + (long)m * (Y + (long)m * Z);
      }
    };
    T *ue = lds, *w1b = ue + kd, *w2b = w1b + w1, *V = w2b + w2, *gx = V + q3, *gy = gx + q3, *gz = gy + q3;
    lane_gather<kd, NT, 16, T>(
        tid,
        [&](int e) {
          bool bnd;
          const T x = a.u[node(e, bnd)];
          return bnd ? T(0) : x;
        },
        [&](int e, T x) { ue[e] = x; });
    PMG_SYNC();
    using PB = PatDense<nq, k>;
    using PD = PatDense<nq, nq>;
    using PBT = PatDense<k, nq>;
    const OneCell cm{cell};
    if constexpr (DIM == 3) {
      contract1<0, k, k, k, PB, NT, false>(tid, ue, w1b, a.qt.B);
      PMG_SYNC();
      contract1<1, nq, k, k, PB, NT, false>(tid, w1b, w2b, a.qt.B);
      PMG_SYNC();
      contract1<2, nq, nq, k, PB, NT, false>(tid, w2b, V, a.qt.B);
      PMG_SYNC();
      contract1<0, nq, nq, nq, PD, NT, false>(tid, V, gx, a.qt.Dq);
      contract1<1, nq, nq, nq, PD, NT, false>(tid, V, gy, a.qt.Dq);
      contract1<2, nq, nq, nq, PD, NT, false>(tid, V, gz, a.qt.Dq);
      PMG_SYNC();
      flux<3, nq, nq, NT>(tid, gx, gy, gz, a.G, cm);
      PMG_SYNC();
      contract1<0, nq, nq, nq, PD, NT, false>(tid, gx, V, a.qt.DqT);
      PMG_SYNC();
      contract1<1, nq, nq, nq, PD, NT, true>(tid, gy, V, a.qt.DqT);
      PMG_SYNC();
      contract1<2, nq, nq, nq, PD, NT, true>(tid, gz, V, a.qt.DqT);
      PMG_SYNC();
      contract1<0, nq, nq, nq, PBT, NT, false>(tid, V, w2b, a.qt.BT);  // (k, nq, nq) fits w2 (nq nq k)
      PMG_SYNC();
      contract1<1, k, nq, nq, PBT, NT, false>(tid, w2b, w1b, a.qt.BT);  // (k, k, nq) fits w1 (nq k k)
      PMG_SYNC();
      contract1<2, k, k, nq, PBT, NT, false>(tid, w1b, ue, a.qt.BT);
    } else {
      contract1<0, k, k, 1, PB, NT, false>(tid, ue, w1b, a.qt.B);
      PMG_SYNC();
      contract1<1, nq, k, 1, PB, NT, false>(tid, w1b, V, a.qt.B);
      PMG_SYNC();
      contract1<0, nq, nq, 1, PD, NT, false>(tid, V, gx, a.qt.Dq);
      contract1<1, nq, nq, 1, PD, NT, false>(tid, V, gy, a.qt.Dq);
      PMG_SYNC();
      flux<2, nq, nq, NT>(tid, gx, gy, gz, a.G, cm);
      PMG_SYNC();
      contract1<0, nq, nq, 1, PD, NT, false>(tid, gx, V, a.qt.DqT);
      PMG_SYNC();
      contract1<1, nq, nq, 1, PD, NT, true>(tid, gy, V, a.qt.DqT);
      PMG_SYNC();
      contract1<0, nq, nq, 1, PBT, NT, false>(tid, V, w1b, a.qt.BT);
      PMG_SYNC();
      contract1<1, k, nq, 1, PBT, NT, false>(tid, w1b, ue, a.qt.BT);
    }
    PMG_SYNC();
    // out += sign * (cell result) on the cell's interior-of-mesh nodes (cells of one color
    // share no node); the loads of out are batched
    lane_gather<kd, NT, 16, T>(
        tid,
        [&](int e) {
          bool bnd;
          return a.out[node(e, bnd)];
        },
        [&](int e, T x) {
          bool bnd;
          const long gi = node(e, bnd);
          if (!bnd) a.out[gi] = x + a.sign * ue[e];
        });
  }
};

// out = b (residual) or 0 (apply) on interior nodes; out = b - u or u on boundary nodes
template <typename T>
PMG_INLINE void metric_apply_init(long g, int dim, int m, bool resid, const T *b, const T *u, T *out) {
  const int i = (int)(g % m), j = (int)((g / m) % m), k = dim == 3 ? (int)(g / ((long)m * m)) : 1;
  const bool bnd = i == 0 || i == m - 1 || j == 0 || j == m - 1 || k == 0 || k == m - 1;
  if (bnd)
    out[g] = resid ? b[g] - u[g] : u[g];
  else
    out[g] = resid ? b[g] : T(0);
}

// the same on a general hex mesh: bnd marks the Dirichlet nodes
template <typename T>
PMG_INLINE void hex_apply_init(long g, bool resid, const unsigned char *bnd, const T *b, const T *u, T *out) {
  if (bnd[g])
    out[g] = resid ? b[g] - u[g] : u[g];
  else
    out[g] = resid ? b[g] : T(0);
}

// ---------------------------------------------------------------------------------------
// Setup: element-matrix diagonals per cell, then patch inverse diagonals (Sec. 3.2: the
// Jacobi smoother of every p-level stores the inverse diagonal of A_{j,p} per patch).
// ---------------------------------------------------------------------------------------
template <int DIM, typename S>
PMG_INLINE void cell_diag(long t, int q, const double *B, const double *Dn, const S *G, double *out) {
  // t = cell * (q+1)^d + node ; diag = sum_g grad_phi^T G grad_phi
  const int k = q + 1, nq = q + 1, kd = DIM == 3 ? k * k * k : k * k, nqd = DIM == 3 ? nq * nq * nq : nq * nq;
  const long cell = t / kd;
  const int node = (int)(t % kd);
  const int a = node % k, b = (node / k) % k, c = DIM == 3 ? node / (k * k) : 0;
  double s = 0.0;
  for (int g = 0; g < nqd; ++g) {
    const int gx = g % nq, gy = (g / nq) % nq, gz = DIM == 3 ? g / (nq * nq) : 0;
    const double bx = B[gx * k + a], by = B[gy * k + b], dx = Dn[gx * k + a], dy = Dn[gy * k + b];
    const long gi = (cell * nqd + g) * (DIM == 3 ? 6 : 3);
    if (DIM == 3) {
      const double bz = B[gz * k + c], dz = Dn[gz * k + c];
      const double p0 = dx * by * bz, p1 = bx * dy * bz, p2 = bx * by * dz;
      const double xx = load_s<double>(G, gi), yy = load_s<double>(G, gi + 1), zz = load_s<double>(G, gi + 2);
      const double xy = load_s<double>(G, gi + 3), xz = load_s<double>(G, gi + 4), yz = load_s<double>(G, gi + 5);
      s += xx * p0 * p0 + yy * p1 * p1 + zz * p2 * p2 + 2.0 * (xy * p0 * p1 + xz * p0 * p2 + yz * p1 * p2);
    } else {
      const double p0 = dx * by, p1 = bx * dy;
      const double xx = load_s<double>(G, gi), yy = load_s<double>(G, gi + 1), xy = load_s<double>(G, gi + 2);
      s += xx * p0 * p0 + yy * p1 * p1 + 2.0 * xy * p0 * p1;
    }
  }
  out[t] = s;
}

// t = patch * (2q-1)^d + e: sum the element diagonals of the cells containing the node and
// store omega / sum in the storage type
template <int DIM, typename S>
PMG_INLINE void patch_inv_diag(long t, int q, int n, double omega, const double *cdiag, S *out) {
  const int e1 = 2 * q - 1, k = q + 1, kd = DIM == 3 ? k * k * k : k * k;
  const long ndp = DIM == 3 ? (long)e1 * e1 * e1 : (long)e1 * e1;
  const long p = t / ndp;
  const int e = (int)(t % ndp);
  const int ii[3] = {e % e1 + 1, (e / e1) % e1 + 1, DIM == 3 ? e / (e1 * e1) + 1 : 0};
  const long k1 = n - 1;
  const int v[3] = {(int)(p % k1) + 1, (int)((p / k1) % k1) + 1, DIM == 3 ? (int)(p / (k1 * k1)) + 1 : 0};
  double s = 0.0;
  const int ncell = 1 << DIM;
  for (int cc = 0; cc < ncell; ++cc) {
    int loc[3] = {0, 0, 0}, cell[3] = {0, 0, 0};
    bool in = true;
    for (int d = 0; d < DIM; ++d) {
      const int side = (cc >> d) & 1;
      const int l = ii[d] - side * q;
      if (l < 0 || l > q) in = false;
      loc[d] = l;
      cell[d] = v[d] - 1 + side;
    }
    if (!in) continue;
    const long cidx = cell[0] + (long)n * (cell[1] + (long)n * (DIM == 3 ? cell[2] : 0));
    const int lidx = loc[0] + k * (loc[1] + k * (DIM == 3 ? loc[2] : 0));
    s += cdiag[cidx * kd + lidx];
  }
  out[t] = to_storage<S>(omega / s);
}

}  // namespace pmg

namespace pmg {
// t = patch * (2q-1)^d + e on a general hex mesh: the patch's cells come from its stored
// list (block position dx + 2 dy + 4 dz); otherwise as patch_inv_diag.
template <int DIM, typename S>
PMG_INLINE void patch_inv_diag_list(long t, int q, const int32_t *pcells, double omega, const double *cdiag, S *out) {
  const int e1 = 2 * q - 1, k = q + 1, kd = DIM == 3 ? k * k * k : k * k;
  const long ndp = DIM == 3 ? (long)e1 * e1 * e1 : (long)e1 * e1;
  const long p = t / ndp;
  const int e = (int)(t % ndp);
  const int ii[3] = {e % e1 + 1, (e / e1) % e1 + 1, DIM == 3 ? e / (e1 * e1) + 1 : 0};
  double s = 0.0;
  const int ncell = 1 << DIM;
  for (int cc = 0; cc < ncell; ++cc) {
    int loc[3] = {0, 0, 0};
    bool in = true;
    for (int d = 0; d < DIM; ++d) {
      const int l = ii[d] - ((cc >> d) & 1) * q;
      if (l < 0 || l > q) in = false;
      loc[d] = l;
    }
    if (!in) continue;
    const long cidx = pcells[p * ncell + cc];
    const int lidx = loc[0] + k * (loc[1] + k * (DIM == 3 ? loc[2] : 0));
    s += cdiag[cidx * kd + lidx];
  }
  out[t] = to_storage<S>(omega / s);
}
}  // namespace pmg
