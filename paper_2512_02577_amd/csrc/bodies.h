// Kernel bodies of the p-multigrid patch smoother library.
//
// Each body is written for one workgroup (threads tid = 0..NT-1, LDS arena `lds`) and
// is __host__ __device__, so that the HIP kernels run it on gfx950 and a CPU build runs
// it with NT = 1 for index and bounds checking.
//
// Discretization on a Cartesian h-level with cell size h (paper Sec. 2 and Sec. 3): the
// operator is c * sum_k K_k (x) M_others with c = h^(dim-2) and K, M the 1D reference
// stiffness and mass matrices of the degree-p Gauss-Lobatto Lagrange basis integrated by
// the (p+1)-point Gauss rule.  All 1D tables come from host_tables.cpp.
#pragma once

#include "sumfac.h"

namespace pmg {

template <typename T>
struct DevTabs {
  const T *Kp[4], *Mp[4], *invD[4], *Tp[4], *TpT[4];  // per p-level, coarsest first
  const T *S[4], *ST[4], *Linv[4];                    // fast diagonalization per p-level > 0
  const T *Kr, *Mr;                                   // patch residual (degree p)
  const T *Kt, *Mt;                                   // apply tile (degree p)
  const T *W1, *Wr;                                   // h-embedding
};

// Workgroup -> work item mapping that keeps consecutive items on one XCD: the hardware
// hands workgroups round-robin to the 8 XCDs, each with its own L2, so item ranges are
// split into 8 contiguous chunks and workgroup b takes item (b / 8) of chunk (b % 8).
PMG_INLINE int xcd_remap(int b, int G) {
  const int per = G / 8, rem = G % 8, x = b % 8, loc = b / 8;
  return x * per + (x < rem ? x : rem) + loc;
}

// ---------------------------------------------------------------------------------------
// Vertex-patch smoother (Alg. 1 body for one patch, Alg. 2 local solve, Alg. 3 p-cycle).
// ---------------------------------------------------------------------------------------
// Damping per p-level, passed by value (indexed with compile-time levels, so it stays in
// registers).
template <typename T>
struct Omega {
  T w[4];
};

template <typename T>
struct SmoothArgs {
  DevTabs<T> tb;
  T c, cinv;         // h^(d-2) and its inverse
  int n;             // cells per direction of this h-level
  int first[3];      // first patch vertex coordinate of the color per axis (1 or 2)
  int cnt[3];        // patches of the color per axis
  int n_patch;       // cnt[0]*cnt[1]*cnt[2]
  int full;          // full V-cycle (post-smoothing) instead of the half V-cycle
  int n_iter;        // Richardson steps of LocalSolve
  int direct;        // LocalSolve is the exact patch solve (fast diagonalization)
  int reinf;         // p-level Richardson preconditioner: Cartesian-reinforced, not Jacobi
  Omega<T> om;       // damping per p-level of the reinforced preconditioner
  T *u;              // solution, updated on patch interiors
  const T *b;        // right-hand side
  // local-solve-only mode (pmg_local_solve): r/d blocks per patch, patch index offset
  const T *r_blocks;
  T *d_blocks;
  int first_patch;
};

template <int... Qs>
struct Degrees {
  static constexpr int L = sizeof...(Qs);
  static constexpr int q[L] = {Qs...};
};

template <int DIM, typename T, int NT, int P, class H>
struct PatchBody {
  static constexpr int L = H::L;
  static_assert(H::q[L - 1] == P, "top p-level must be the degree");
  static_assert(H::q[0] == 1, "coarsest p-level must be degree 1");
  static constexpr int N = 2 * P + 1, n = 2 * P - 1;
  static constexpr int Nd = ipow(N, DIM), nd = ipow(n, DIM);
  static constexpr int qd(int l) { return H::q[l]; }
  static constexpr int nl(int l) { return 2 * H::q[l] - 1; }
  static constexpr int ndl(int l) { return ipow(2 * H::q[l] - 1, DIM); }

  // ---- LDS layout (every contraction that shrinks a tensor runs in place) ----
  // phase R (patch residual): r | closure tensor (2D) or Zm = Mz u (3D; stage outputs in
  //                           place) | B (2D) or Zk = Kz u (3D)
  // phase S (local solve):    r | d | partial sums | r_l, d_l of levels L-2 .. 1 | X (2 nd) | cc
  // X holds a level's vmult pair (A, B; the residual lands on A in place), the in-place
  // restriction of that residual, and the two stages of a prolongation.  cc (the
  // correction of Richardson steps after the first) is at the end, so that one step
  // needs only `size1`.
  // One half V-cycle alone (the default local solver's own kernels, ONE) reads r last in
  // the top level's residual; the lower levels' r_l, d_l then take r's place when they
  // fit there (layout A):  r, later r_l, d_l of levels L-2 .. 1 | d | partial sums | X.
  static constexpr int off_r = 0;  // patch residual, then running Richardson residual
  static constexpr int off_ucl = nd;
  static constexpr int off_B = nd + (DIM == 3 ? n * N * N : Nd);
  static constexpr int phaseR_end = off_B + (DIM == 3 ? n * N * N : n * N);
  static constexpr int off_d = nd;
  static constexpr int NRED = 8;  // per-wave partial sums of block_sum (up to 8 waves)
  static constexpr int off_red = 2 * nd;
  static constexpr int lower_size(int l) { return l <= 0 ? 0 : 2 * ndl(l) + lower_size(l - 1); }  // levels 1..l
  static constexpr int off_lr(int l) { return 2 * nd + NRED + lower_size(l - 1); }
  static constexpr int off_ld(int l) { return off_lr(l) + ndl(l); }
  static constexpr int off_X = 2 * nd + NRED + lower_size(L - 2);
  static constexpr int phaseS_end = off_X + 2 * nd;
  static constexpr int size1 = cmax(phaseR_end, phaseS_end);
  static constexpr int off_cc = size1;
  static constexpr int size = size1 + nd;
  static constexpr bool ALIAS = lower_size(L - 2) <= nd;  // layout A possible
  template <bool A>
  static constexpr int offX() { return A ? 2 * nd + NRED : off_X; }
  template <bool A>
  static constexpr int offLR(int l) { return A ? lower_size(l - 1) : off_lr(l); }
  template <bool A>
  static constexpr int offLD(int l) { return offLR<A>(l) + ndl(l); }
  // arena of the ONE kernels
  static constexpr int size_one = ALIAS ? cmax(phaseR_end, offX<true>() + 2 * nd) : size1;
  static_assert(NT <= 64 * NRED, "block_sum scratch");

  // res = r - c A_l d on p-level l (interior patch operator); A, B scratch in X, res may
  // be X itself (the last stage lands on A in place) or r
  template <int l, bool AL = false>
  PMG_INLINE static void vmult_residual(int tid, T *lds, const DevTabs<T> &tb, T c, const T *d, const T *r,
                                        T *res) {
    constexpr int m = nl(l);
    using Pat = PatInterior<qd(l)>;
    using D = Dense<m, m>;
    T *A = lds + offX<AL>(), *B = lds + offX<AL>() + ndl(l);
    if constexpr (DIM == 3) {
      scontract2<0, m, m, m, Pat, NT, D, D, D>(tid, d, A, tb.Mp[l], B, tb.Kp[l]);  // A = Mx d, B = Kx d
      PMG_SYNC();
      scontract_pair<1, m, m, m, Pat, NT, D, D>(tid, A, B, tb.Mp[l], tb.Kp[l]);  // C = My A, G = Ky A + My B
      PMG_SYNC();
      scontract_final<2, m, m, m, Pat, NT, D, D, D, true>(tid, A, B, res, r, c, tb.Kp[l], tb.Mp[l]);
    } else {
      scontract2<0, m, m, 1, Pat, NT, D, D, D>(tid, d, A, tb.Mp[l], B, tb.Kp[l]);
      PMG_SYNC();
      scontract_final<1, m, m, 1, Pat, NT, D, D, D, true>(tid, A, B, res, r, c, tb.Kp[l], tb.Mp[l]);
    }
  }

  PMG_INLINE static void decode_l(int e, int m, int k[3]) {
    k[0] = e % m;
    k[1] = (e / m) % m;
    k[2] = DIM == 3 ? e / (m * m) : 0;
  }

  // Alg. 3 on p-level l: d = V(l, r), zero initial guess.
  // Inverse diagonals of the top p-level and of p-level 1 read ahead into registers (with the
  // patch gathers), so that the local solve does not wait for them; only where they fit a
  // few registers per lane.
  static constexpr int RPT = (nd + NT - 1) / NT;
  static constexpr int RP1 = L >= 3 ? (ndl(1) + NT - 1) / NT : 1;
  static constexpr bool PRE_T = RPT <= 4, PRE_1 = L >= 3 && RP1 <= 2;
  struct PreD {
    T top[PRE_T ? RPT : 1];
    T l1[PRE_1 ? RP1 : 1];
  };

  PMG_INLINE static void prefetch_diag(int tid, const DevTabs<T> &tb, PreD &pre) {
    if constexpr (PRE_T) {
      const cptr<T> iv = as_const(tb.invD[L - 1]);
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int e = tid + j * NT;
        pre.top[j] = iv[e < nd ? e : nd - 1];
      }
    }
    if constexpr (PRE_1) {
      constexpr int n1 = ndl(1);
      const cptr<T> iv = as_const(tb.invD[1]);
#pragma unroll
      for (int j = 0; j < RP1; ++j) {
        const int e = tid + j * NT;
        pre.l1[j] = iv[e < n1 ? e : n1 - 1];
      }
    }
  }

  // d = cinv D_l^-1 r on p-level l, from the read-ahead diagonal when there is one
  template <int l>
  PMG_INLINE static void jacobi(int tid, const DevTabs<T> &tb, T cinv, const T *r, T *d, const PreD *pre) {
    constexpr int ndq = ndl(l);
    constexpr bool HAVE = (l == L - 1 && PRE_T) || (l == 1 && PRE_1);
    if (HAVE && pre) {
      constexpr int R = (ndq + NT - 1) / NT;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int e = tid + j * NT;
        const T x = l == L - 1 ? pre->top[j < RPT ? j : 0] : pre->l1[j < RP1 ? j : 0];
        if (e < ndq) d[e] = cinv * x * r[e];
      }
    } else {
      const cptr<T> invD = as_const(tb.invD[l]);
      lane_gather<ndq, NT, 16, T>(tid, [&](int e) { return invD[e]; }, [&](int e, T x) { d[e] = cinv * x * r[e]; });
    }
  }

  // d = s (S x S x S) diag(Linv) (S x S x S)^T r on p-level l >= 1: fast diagonalization of
  // the interior patch operator c sum_k K_k (x) M_others (K S = M S diag(lam), S^T M S = I),
  // its inverse for s = 1/c.  Dense 1D contractions, the first from r into d, the others in
  // place on d (r and d distinct, ndl(l) entries each).
  template <int l>
  PMG_INLINE static void fdm(int tid, const DevTabs<T> &tb, T s, const T *r, T *d) {
    constexpr int m = nl(l);
    using Pat = PatDense<m, m>;
    using D = Dense<m, m>;
    if constexpr (DIM == 3) {
      scontract1<0, m, m, m, Pat, NT, false, D, D>(tid, r, d, tb.ST[l]);
      PMG_SYNC();
      scontract1<1, m, m, m, Pat, NT, false, D, D, true>(tid, d, d, tb.ST[l]);
      PMG_SYNC();
      scontract1<2, m, m, m, Pat, NT, false, D, D, true>(tid, d, d, tb.ST[l]);
    } else {
      scontract1<0, m, m, 1, Pat, NT, false, D, D>(tid, r, d, tb.ST[l]);
      PMG_SYNC();
      scontract1<1, m, m, 1, Pat, NT, false, D, D, true>(tid, d, d, tb.ST[l]);
    }
    PMG_SYNC();
    const cptr<T> Li = as_const(tb.Linv[l]);
    for (int e = tid; e < ndl(l); e += NT) d[e] *= s * Li[e];
    PMG_SYNC();
    if constexpr (DIM == 3) {
      scontract1<0, m, m, m, Pat, NT, false, D, D, true>(tid, d, d, tb.S[l]);
      PMG_SYNC();
      scontract1<1, m, m, m, Pat, NT, false, D, D, true>(tid, d, d, tb.S[l]);
      PMG_SYNC();
      scontract1<2, m, m, m, Pat, NT, false, D, D, true>(tid, d, d, tb.S[l]);
    } else {
      scontract1<0, m, m, 1, Pat, NT, false, D, D, true>(tid, d, d, tb.S[l]);
      PMG_SYNC();
      scontract1<1, m, m, 1, Pat, NT, false, D, D, true>(tid, d, d, tb.S[l]);
    }
  }

  // reinf: the p-level Richardson steps use the Cartesian-reinforced preconditioner (on the
  // Cartesian path the inverse of the patch operator by fast diagonalization, damped by
  // om[l]) instead of damped Jacobi
  // AL: layout A (one half V-cycle alone; r is not read after this level's residual)
  template <int l, bool AL = false>
  PMG_INLINE static void cycle(int tid, T *lds, const DevTabs<T> &tb, T c, T cinv, const T *r, T *d,
                               bool full, const PreD *pre = nullptr, bool reinf = false,
                               Omega<T> om = Omega<T>{}) {
    if constexpr (l == 0) {
      if (tid == 0) d[0] = cinv * as_const(tb.invD[0])[0] * r[0];  // exact 1x1 solve
      PMG_SYNC();
    } else {
      constexpr int q = qd(l), qc = qd(l - 1), m = nl(l), mc = nl(l - 1), ndq = ndl(l);
      const cptr<T> invD = as_const(tb.invD[l]);
      if (reinf)
        fdm<l>(tid, tb, cinv * om.w[l], r, d);  // pre-smoothing d = om P^-1 r
      else
        jacobi<l>(tid, tb, cinv, r, d, pre);  // pre-smoothing d = cinv D^-1 r
      // on p-level 1 the weights of the one-node coarsest level are read now, so that their
      // loads overlap the residual below
      constexpr int R1 = l == 1 ? (ndq + NT - 1) / NT : 1;
      T wp[R1], tp[R1];
      if constexpr (l == 1) {
        const cptr<T> w = as_const(tb.TpT[l]), t = as_const(tb.Tp[l]);
#pragma unroll
        for (int j = 0; j < R1; ++j) {
          const int e = tid + j * NT;
          int k[3];
          decode_l(e < ndq ? e : ndq - 1, m, k);
          wp[j] = w[k[0]] * w[k[1]] * (DIM == 3 ? w[k[2]] : T(1));
          tp[j] = t[k[0]] * t[k[1]] * (DIM == 3 ? t[k[2]] : T(1));
        }
      }
      PMG_SYNC();
      T *res = lds + offX<AL>();
      vmult_residual<l, AL>(tid, lds, tb, c, d, r, res);  // res = r - A d
      PMG_SYNC();
      if constexpr (l == 1) {
        // the coarsest p-level has one node: restriction is a weighted sum, its exact
        // solve a scalar, and prolongation the outer product of the embedding column
        T part = 0;
#pragma unroll
        for (int j = 0; j < R1; ++j) {
          const int e = tid + j * NT;
          if (e < ndq) part += wp[j] * res[e];
        }
        const T r0 = block_sum<NT>(tid, part, lds + off_red);
        const T d0 = cinv * as_const(tb.invD[0])[0] * r0;
#pragma unroll
        for (int j = 0; j < R1; ++j) {
          const int e = tid + j * NT;
          if (e < ndq) d[e] += tp[j] * d0;
        }
        PMG_SYNC();
      } else {
        using PR = PatRestrict<q, qc>;
        using PP = PatProlong<q, qc>;
        using D = Dense<m, m>;
        using DC = Dense<mc, mc>;
        T *rc = lds + offLR<AL>(l - 1), *dc = lds + offLD<AL>(l - 1);
        T *X0 = lds + offX<AL>(), *X1 = lds + offX<AL>() + nd;
        if constexpr (DIM == 3) {
          scontract1<0, m, m, m, PR, NT, false, D, D, true>(tid, res, res, tb.TpT[l]);
          PMG_SYNC();
          scontract1<1, mc, m, m, PR, NT, false, D, D, true>(tid, res, res, tb.TpT[l]);
          PMG_SYNC();
          scontract1<2, mc, mc, m, PR, NT, false, D, DC>(tid, res, rc, tb.TpT[l]);
        } else {
          scontract1<0, m, m, 1, PR, NT, false, D, D, true>(tid, res, res, tb.TpT[l]);
          PMG_SYNC();
          scontract1<1, mc, m, 1, PR, NT, false, D, DC>(tid, res, rc, tb.TpT[l]);
        }
        PMG_SYNC();
        cycle<l - 1, AL>(tid, lds, tb, c, cinv, rc, dc, full, pre, reinf, om);
        if constexpr (DIM == 3) {  // d += P dc
          scontract1<0, mc, mc, mc, PP, NT, false, DC, Dense<m, mc>>(tid, dc, X0, tb.Tp[l]);
          PMG_SYNC();
          scontract1<1, m, mc, mc, PP, NT, false, Dense<m, mc>, D>(tid, X0, X1, tb.Tp[l]);
          PMG_SYNC();
          scontract1<2, m, m, mc, PP, NT, true, D, D>(tid, X1, d, tb.Tp[l]);
        } else {
          scontract1<0, mc, mc, 1, PP, NT, false, DC, Dense<m, mc>>(tid, dc, X0, tb.Tp[l]);
          PMG_SYNC();
          scontract1<1, m, mc, 1, PP, NT, true, Dense<m, mc>, D>(tid, X0, d, tb.Tp[l]);
        }
        PMG_SYNC();
      }
      if (!AL && full) {  // post-smoothing (layout A has overwritten r: half V-cycles only)
        vmult_residual<l, AL>(tid, lds, tb, c, d, r, res);
        PMG_SYNC();
        if (reinf) {
          T *tmp = res + ndq;  // the vmult's second stage buffer, dead now
          fdm<l>(tid, tb, cinv * om.w[l], res, tmp);
          PMG_SYNC();
          for (int e = tid; e < ndq; e += NT) d[e] += tmp[e];
        } else {
          lane_gather<ndq, NT, 16, T>(
              tid, [&](int e) { return invD[e]; }, [&](int e, T x) { d[e] += cinv * x * res[e]; });
        }
        PMG_SYNC();
      }
    }
  }

  // Alg. 2: d = LocalSolve(r) on the top level (r at off_r, d at off_d).  Later Richardson
  // steps keep a running residual r <- r - A c, equal to r_0 - A d.  ONE: the local solver is
  // one half V-cycle (the default), compiled without the code of the other variants.
  template <bool ONE = false>
  PMG_INLINE static void local_solve(int tid, T *lds, const SmoothArgs<T> &a, const PreD *pre = nullptr) {
    T *r = lds + off_r, *d = lds + off_d, *cc = lds + off_cc;
    if constexpr (ONE) {
      cycle<L - 1, ALIAS>(tid, lds, a.tb, a.c, a.cinv, r, d, false, pre);
      return;
    }
    if constexpr (L >= 2) {
      if (a.direct) {  // exact patch solve: d = A_j^-1 r
        fdm<L - 1>(tid, a.tb, a.cinv, r, d);
        PMG_SYNC();
        return;
      }
    }
    const bool full = a.full != 0, reinf = a.reinf != 0;
    cycle<L - 1>(tid, lds, a.tb, a.c, a.cinv, r, d, full, nullptr, reinf, a.om);
    for (int it = 1; it < a.n_iter; ++it) {
      vmult_residual<L - 1>(tid, lds, a.tb, a.c, it == 1 ? d : cc, r, r);
      PMG_SYNC();
      cycle<L - 1>(tid, lds, a.tb, a.c, a.cinv, r, cc, full, nullptr, reinf, a.om);
      for (int e = tid; e < nd; e += NT) d[e] += cc[e];
      PMG_SYNC();
    }
  }

  // Arena elements for n_iter Richardson steps, and of the ONE kernels.
  PMG_HD static constexpr int arena(int n_iter) { return n_iter > 1 ? size : size1; }
  PMG_HD static constexpr int arena_one() { return size_one; }

  PMG_INLINE static void decode(int idx, int k[3]) {
    k[0] = idx % n;
    k[1] = (idx / n) % n;
    k[2] = DIM == 3 ? idx / (n * n) : 0;
  }

  // One patch of one color: gather, residual, LocalSolve, scatter (Alg. 1 body).
  template <bool ONE = false>
  PMG_INLINE static void smooth_patch(int tid, int blk, T *lds, const SmoothArgs<T> &a) {
    const int pidx = xcd_remap(blk, a.n_patch);
    int v[3];
    v[0] = a.first[0] + 2 * (pidx % a.cnt[0]);
    v[1] = a.first[1] + 2 * ((pidx / a.cnt[0]) % a.cnt[1]);
    v[2] = DIM == 3 ? a.first[2] + 2 * (pidx / (a.cnt[0] * a.cnt[1])) : 0;
    const int m = P * a.n + 1;
    const int g0[3] = {P * (v[0] - 1), P * (v[1] - 1), DIM == 3 ? P * (v[2] - 1) : 0};
    T *ucl = lds + off_ucl, *r = lds + off_r;
    const T *__restrict__ u_in = a.u;
    // The patch interior of u is written only by this patch while its color runs (no
    // other patch of the color has it in its closure), so the values the final update
    // adds to can be read now, with the gathers, instead of after the local solve.
    PreD pre;
    if constexpr (ONE) prefetch_diag(tid, a.tb, pre);
    constexpr int NUI = (nd + NT - 1) / NT;
    constexpr bool KEEP = NUI <= 3;
    T uold[KEEP ? NUI : 1];
    if constexpr (KEEP) {
#pragma unroll
      for (int k = 0; k < NUI; ++k) {
        const int e = tid + k * NT;
        uold[k] = u_in[interior_index(e < nd ? e : nd - 1, g0, m)];
      }
    }
    const T *__restrict__ b_in = a.b;
    using Pat = PatResidual<P>;
    if constexpr (DIM == 3) {
      // r = b - c (sum_k Kr_k (x) Mr_others) ubar, the z contraction first: a lane per closure
      // column (i, j) loads its N nodes from global memory (zero on the Dirichlet boundary;
      // every closure node lies inside the mesh, so the load is always valid) and writes
      // Zm = Mr_z ubar and Zk = Kr_z ubar at the n interior planes; the closure itself never
      // goes through LDS.  Then y (in place) and x (into r, on top of b).
      T *Zm = ucl, *Zk = lds + off_B;
      const cptr<T> Mr0 = as_const(a.tb.Mr), Kr0 = as_const(a.tb.Kr);
      // the column as loaded; the Dirichlet mask is applied where it is used, so that the loads
      // stay in flight over the gather of b
      auto load_col = [&](int col, T *w) {
        const T *cp = u_in + ((g0[0] + col % N) + m * ((g0[1] + col / N) + m * g0[2]));
#pragma unroll
        for (int k = 0; k < N; ++k) w[k] = cp[m * m * k];
      };
      auto zstage = [&](int col, T *w) {
        const int gx = g0[0] + col % N, gy = g0[1] + col / N;
        const bool bxy = gx == 0 || gx == m - 1 || gy == 0 || gy == m - 1;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const int gz = g0[2] + k;
          w[k] = (bxy || gz == 0 || gz == m - 1) ? T(0) : w[k];
        }
        const cptr<T> Mr = per_pencil(Mr0), Kr = per_pencil(Kr0);
#pragma unroll
        for (int o = 0; o < n; ++o) {
          Zm[col + N * N * o] = row1<Pat>(Mr, o, w);
          Zk[col + N * N * o] = row1<Pat>(Kr, o, w);
        }
      };
      auto gather_b = [&]() {
        lane_gather<nd, NT, 16, T>(
            tid, [&](int e) { return b_in[interior_index(e, g0, m)]; }, [&](int e, T x) { r[e] = x; });
      };
      if constexpr (NT >= N * N) {
        // one column per lane: its loads are in flight together with those of b
        T w[N];
        load_col(tid < N * N ? tid : N * N - 1, w);
        gather_b();
        if (tid < N * N) zstage(tid, w);
      } else {
        gather_b();
        for (int col = tid; col < N * N; col += NT) {
          T w[N];
          load_col(col, w);
          zstage(col, w);
        }
      }
      PMG_SYNC();
      scontract_pair<1, N, N, n, Pat, NT, Dense<N, N>, Dense<N, N>>(tid, Zm, Zk, a.tb.Mr, a.tb.Kr);
      PMG_SYNC();
      scontract_final<0, N, n, n, Pat, NT, Dense<N, N>, Dense<N, N>, Dense<n, n>>(tid, Zm, Zk, r, r, a.c, a.tb.Kr,
                                                                                  a.tb.Mr);
    } else {
      // closure of u (zero on the Dirichlet boundary; every closure node lies inside the
      // mesh, so the load itself is always valid) and the interior of b
      lane_gather2<Nd, nd, NT, 16, T>(
          tid,
          [&](int e) {
            const int i = e % N, j = e / N;
            const int gx = g0[0] + i, gy = g0[1] + j;
            const bool bnd = gx == 0 || gx == m - 1 || gy == 0 || gy == m - 1;
            const T x = u_in[gx + m * gy];
            return bnd ? T(0) : x;
          },
          [&](int e, T x) { ucl[e] = x; }, [&](int e) { return b_in[interior_index(e, g0, m)]; },
          [&](int e, T x) { r[e] = x; });
      PMG_SYNC();
      // r = b - c (sum_k Kr_k (x) Mr_others) ubar   (closure -> interior)
      using DU = Dense<N, N>;
      using DB = Dense<n, N>;
      T *Bb = lds + off_B;
      scontract2<0, N, N, 1, Pat, NT, DU, DU, DB, true>(tid, ucl, ucl, a.tb.Mr, Bb, a.tb.Kr);
      PMG_SYNC();
      scontract_final<1, n, N, 1, Pat, NT, DU, DB, Dense<n, n>>(tid, ucl, Bb, r, r, a.c, a.tb.Kr, a.tb.Mr);
    }
    PMG_SYNC();
    local_solve<ONE>(tid, lds, a, ONE ? &pre : nullptr);
    const T *d = lds + off_d;
    if constexpr (KEEP) {
#pragma unroll
      for (int k = 0; k < NUI; ++k) {
        const int e = tid + k * NT;
        if (e < nd) a.u[interior_index(e, g0, m)] = uold[k] + d[e];
      }
    } else {
      lane_gather<nd, NT, 16, T>(
          tid, [&](int e) { return a.u[interior_index(e, g0, m)]; },
          [&](int e, T x) { a.u[interior_index(e, g0, m)] = x + d[e]; });
    }
  }

  // global index of patch-interior element e of the patch whose closure starts at g0
  PMG_INLINE static int interior_index(int e, const int g0[3], int m) {
    int k[3];
    decode(e, k);
    return (g0[0] + 1 + k[0]) + m * ((g0[1] + 1 + k[1]) + m * (g0[2] + (DIM == 3 ? 1 : 0) + k[2]));
  }

  // LocalSolve alone on block blk of r_blocks -> d_blocks
  PMG_INLINE static void local_only(int tid, int blk, T *lds, const SmoothArgs<T> &a) {
    T *r = lds + off_r;
    const size_t base = (size_t)blk * nd;
    lane_gather<nd, NT, 16, T>(tid, [&](int e) { return a.r_blocks[base + e]; }, [&](int e, T x) { r[e] = x; });
    PMG_SYNC();
    local_solve(tid, lds, a);
    const T *d = lds + off_d;
    for (int e = tid; e < nd; e += NT) a.d_blocks[base + e] = d[e];
  }
};

// ---------------------------------------------------------------------------------------
// Operator apply v = A u (or residual r = b - A u) on a Cartesian h-level.  A tile of TC^d
// cells owns the nodes P*c0 .. P*(c0+TC)-1 per direction (plus the last node of the mesh
// for tiles at the upper end); it reads the nodes of its cells and of one extra cell below,
// so every owned node sees all of its cells and each output is written by one workgroup.
// ---------------------------------------------------------------------------------------
template <typename T>
struct ApplyArgs {
  const T *Kt, *Mt;
  T c;
  int n;       // cells per direction
  int ntile;   // tiles per direction
  int n_tiles; // total tiles (workgroups)
  int mt, mty, zc;  // marching apply: tiles in x and in y, cell layers per z segment
  const T *u;
  const T *b;  // residual mode
  T *out;
};

// MASS: v = c (M (x) M (x) M) u instead, the consistent mass matrix (c = h^d), with zero rows
// and columns on the Dirichlet boundary.
template <int DIM, typename T, int NT, int P, int TC, bool RESID, bool MASS = false>
struct ApplyBody {
  static_assert(!(RESID && MASS), "the mass apply has no residual form");
  static constexpr int NI = P * (TC + 1) + 1, NO = P * TC;
  static constexpr int NId = ipow(NI, DIM), NOd = ipow(NO, DIM);
  using RS = LapScratch<DIM, NI, NO>;
  static constexpr int R0 = cmax(NId, RS::cg);
  static constexpr int R1 = RS::ab;
  static_assert(DIM == 2 ? NOd <= R0 : NOd <= R1, "output tile must fit its overlay");
  static constexpr int size = R0 + R1;

  PMG_INLINE static void run(int tid, int blk, T *lds, const ApplyArgs<T> &a) {
    const int t = xcd_remap(blk, a.n_tiles);
    const int tt[3] = {t % a.ntile, (t / a.ntile) % a.ntile, DIM == 3 ? t / (a.ntile * a.ntile) : 0};
    const int m = P * a.n + 1;
    int c0[3], lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      c0[d] = TC * tt[d];
      lo[d] = P * (c0[d] - 1);                       // first input node
      hi[d] = (c0[d] + TC >= a.n) ? m : P * (c0[d] + TC);  // one past the last owned node
    }
    // the output tile overlays whatever is dead when the last stage writes it: ab in 3D
    // (read by stage 2 only), the input tile in 2D (read by stage 1 only)
    T *in = lds, *ab = lds + R0, *outl = DIM == 3 ? lds + R0 : lds;
    if constexpr (DIM == 3) {
      run3(tid, a, m, c0, lo, hi, in, ab, outl);
      return;
    }
    const T *__restrict__ u = a.u;
    // owned outputs: bx x by x bz nodes from P*c0 (one more per direction at the upper end)
    const int bx = hi[0] - P * c0[0], by = hi[1] - P * c0[1], bz = DIM == 3 ? hi[2] - P * c0[2] : 1;
    const int tot = bx * by * bz;
    auto out_index = [&](int e, bool &bnd) {
      const int ox = e % bx, oy = (e / bx) % by, oz = DIM == 3 ? e / (bx * by) : 0;
      const int gx = P * c0[0] + ox, gy = P * c0[1] + oy, gz = DIM == 3 ? P * c0[2] + oz : 0;
      bnd = gx == 0 || gx == m - 1 || gy == 0 || gy == m - 1;
      if (DIM == 3) bnd = bnd || gz == 0 || gz == m - 1;
      return gx + m * (gy + m * gz);
    };
    // b and the boundary values of u at the owned outputs are read up front, with the input
    // tile, when they fit a few registers per lane; otherwise in groups at the end
    constexpr int NOm = ipow(NO + 1, DIM), RO = (NOm + NT - 1) / NT;
    constexpr bool PRE = RO <= 8;
    T ub[PRE ? RO : 1], bb[PRE ? RO : 1];
    if constexpr (PRE) {
#pragma unroll
      for (int k = 0; k < RO; ++k) {
        const int e = tid + k * NT;
        bool bnd;
        const int gi = out_index(e < tot ? e : tot - 1, bnd);
        ub[k] = u[gi];
        if (RESID) bb[k] = a.b[gi];
      }
    }
    // input tile: nodes outside the mesh or on its boundary are zero (the load address is
    // clamped into the mesh and the value dropped)
    lane_gather<NId, NT, 24, T>(
        tid,
        [&](int e) {
          const int i = e % NI, j = (e / NI) % NI, k = DIM == 3 ? e / (NI * NI) : 0;
          const int gx = lo[0] + i, gy = lo[1] + j, gz = DIM == 3 ? lo[2] + k : 0;
          bool ok = gx > 0 && gx < m - 1 && gy > 0 && gy < m - 1;
          if (DIM == 3) ok = ok && gz > 0 && gz < m - 1;
          const int cx = gx < 0 ? 0 : (gx > m - 1 ? m - 1 : gx);
          const int cy = gy < 0 ? 0 : (gy > m - 1 ? m - 1 : gy);
          const int cz = gz < 0 ? 0 : (gz > m - 1 ? m - 1 : gz);
          const T x = u[cx + m * (cy + m * cz)];
          return ok ? x : T(0);
        },
        [&](int e, T x) { in[e] = x; });
    PMG_SYNC();
    if constexpr (MASS)
      kron_all<DIM, PatTile<P, TC>, NT, false>(tid, in, outl, a.Mt, ab, (T *)nullptr);
    else
      laplace_sf<DIM, PatTile<P, TC>, NT>(tid, in, outl, (const T *)nullptr, a.c, a.Kt, a.Mt, ab, in);
    PMG_SYNC();
    auto finish = [&](int e, T uv, T bv) {
      bool bnd;
      const int gi = out_index(e, bnd);
      const int ox = e % bx, oy = (e / bx) % by, oz = DIM == 3 ? e / (bx * by) : 0;
      T val = bnd ? uv : outl[ox + NO * (oy + NO * oz)];
      if (MASS) val = bnd ? T(0) : a.c * val;
      if (RESID) val = bv - val;
      a.out[gi] = val;
    };
    if constexpr (PRE) {
#pragma unroll
      for (int k = 0; k < RO; ++k) {
        const int e = tid + k * NT;
        if (e < tot) finish(e, ub[k], RESID ? bb[k] : T(0));
      }
    } else {
      constexpr int G = 8;
      for (int k0 = 0; k0 < RO; k0 += G) {
        T uu[G], vb[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
          const int e = tid + (k0 + k) * NT;
          bool bnd;
          const int gi = out_index(e < tot ? e : tot - 1, bnd);
          uu[k] = u[gi];
          vb[k] = RESID ? a.b[gi] : T(0);
        }
#pragma unroll
        for (int k = 0; k < G; ++k) {
          const int e = tid + (k0 + k) * NT;
          if (e < tot) finish(e, uu[k], vb[k]);
        }
      }
    }
  }

  // 3D: the tile is read and written as columns along z.  Each lane owns columns (i, j) and
  // walks k with a running address, so the index arithmetic is done once per column and the
  // per-plane tests (the same on every lane) are scalar.
  PMG_INLINE static void run3(int tid, const ApplyArgs<T> &a, int m, const int c0[3], const int lo[3],
                              const int hi[3], T *in, T *ab, T *outl) {
    const T *__restrict__ u = a.u;
    const int m2 = m * m;
    constexpr int LP = NT < 64 ? NT : 64, NW = NT / LP;  // lanes per wave, waves
    constexpr int NO1 = NO + 1;
    // ---- owned outputs: columns (ox, oy) of bx x by, LP per pass; each wave a range of oz
    const int bx = hi[0] - P * c0[0], by = hi[1] - P * c0[1], bz = hi[2] - P * c0[2];
    const int bxy = bx * by;
    constexpr int QC = (NO1 * NO1 + LP - 1) / LP, ZS = (NO1 + NW - 1) / NW;
    const int lane = tid % LP, w = tid / LP;
    const int zs = (bz + NW - 1) / NW, z0 = w * zs;
    int gcol[QC], lcol[QC];
    bool bxyc[QC];
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      int e2 = lane + LP * q;
      e2 = e2 < bxy ? e2 : bxy - 1;
      const int ox = e2 % bx, oy = e2 / bx;
      const int gx = P * c0[0] + ox, gy = P * c0[1] + oy;
      bxyc[q] = gx == 0 || gx == m - 1 || gy == 0 || gy == m - 1;
      gcol[q] = gx + m * gy;
      lcol[q] = ox + NO * oy;
    }
    auto zidx = [&](int z) {  // owned plane of slot z (clamped)
      const int oz = z0 + z;
      return oz < bz ? oz : bz - 1;
    };
    // ---- input tile: NI^2 columns of NI nodes; nodes outside the mesh or on its boundary are
    // zero (the load address is clamped into the mesh and the value dropped).  QG columns per
    // lane are in flight together.
    constexpr int NC = NI * NI, QI = (NC + NT - 1) / NT, QG = NI * 2 <= 32 ? 2 : 1;
#pragma unroll
    for (int q0 = 0; q0 < QI; q0 += QG) {
      T v[QG][NI];
      int e2s[QG];
#pragma unroll
      for (int g = 0; g < QG; ++g) {
        int e2 = tid + (q0 + g) * NT;
        e2s[g] = e2;
        e2 = e2 < NC ? e2 : NC - 1;
        const int i = e2 % NI, j = e2 / NI;
        const int gx = lo[0] + i, gy = lo[1] + j;
        const bool okxy = gx > 0 && gx < m - 1 && gy > 0 && gy < m - 1;
        const int cx = gx < 0 ? 0 : (gx > m - 1 ? m - 1 : gx);
        const int cy = gy < 0 ? 0 : (gy > m - 1 ? m - 1 : gy);
        const T *col = u + (cx + m * cy);
#pragma unroll
        for (int k = 0; k < NI; ++k) {
          const int gz = lo[2] + k;
          const bool ok = okxy && gz > 0 && gz < m - 1;
          const int cz = gz < 0 ? 0 : (gz > m - 1 ? m - 1 : gz);
          const T x = col[m2 * cz];
          v[g][k] = ok ? x : T(0);
        }
      }
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
      for (int g = 0; g < QG; ++g)
#pragma unroll
        for (int k = 0; k < NI; ++k) asm volatile("" : "+v"(v[g][k]));
#endif
#pragma unroll
      for (int g = 0; g < QG; ++g)
        if (q0 + g < QI && e2s[g] < NC) {
#pragma unroll
          for (int k = 0; k < NI; ++k) in[e2s[g] + NC * k] = v[g][k];
        }
    }
    PMG_SYNC();
    // the three stages of the tile operator (as laplace_sf: A = Mx u, B = Kx u; C = My A,
    // G = Ky A + My B in the dead input tile; out = c (Kz C + Mz G))
    using Pat = PatTile<P, TC>;
    constexpr int SA = NO * NI * NI, SC = NO * NO * NI;
    if constexpr (MASS) {  // A = Mx u; C = My A
      contract1<0, NI, NI, NI, Pat, NT, false>(tid, in, ab, a.Mt);
      PMG_SYNC();
      contract1<1, NO, NI, NI, Pat, NT, false>(tid, ab, in, a.Mt);
    } else {
      contract2<0, NI, NI, NI, Pat, NT>(tid, in, ab, a.Mt, ab + SA, a.Kt);
      PMG_SYNC();
      contract_pair<1, NO, NI, NI, Pat, NT>(tid, ab, ab + SA, in, in + SC, a.Mt, a.Kt);
    }
    PMG_SYNC();
    // b, and u where an owned node is on the mesh boundary (only tiles at the mesh faces have
    // such nodes), are read here so that their loads overlap the last stage, where the
    // fewest registers are live
    const bool edge = c0[0] == 0 || c0[1] == 0 || c0[2] == 0 || hi[0] == m || hi[1] == m || hi[2] == m;
    T bb[RESID ? QC : 1][RESID ? ZS : 1], ub[QC][ZS];
    if constexpr (RESID) {
#pragma unroll
      for (int q = 0; q < QC; ++q)
#pragma unroll
        for (int z = 0; z < ZS; ++z) bb[q][z] = a.b[gcol[q] + m2 * (P * c0[2] + zidx(z))];
    }
    if (edge) {
#pragma unroll
      for (int q = 0; q < QC; ++q)
#pragma unroll
        for (int z = 0; z < ZS; ++z) ub[q][z] = u[gcol[q] + m2 * (P * c0[2] + zidx(z))];
    }
    if constexpr (MASS)
      contract1<2, NO, NO, NI, Pat, NT, false>(tid, in, outl, a.Mt);  // Mz C
    else
      contract_final<2, NO, NO, NI, Pat, NT>(tid, in, in + SC, outl, (const T *)nullptr, a.c, a.Kt, a.Mt);
    PMG_SYNC();
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      if (lane + LP * q >= bxy) continue;
#pragma unroll
      for (int z = 0; z < ZS; ++z) {
        const int oz = z0 + z;
        if (z >= zs || oz >= bz) continue;
        const int gz = P * c0[2] + oz;
        const bool bnd = bxyc[q] || gz == 0 || gz == m - 1;
        T val = outl[lcol[q] + NO * NO * oz];
        if constexpr (MASS) {
          val = (edge && bnd) ? T(0) : a.c * val;
        } else {
          if (edge && bnd) val = ub[q][z];
        }
        if constexpr (RESID) val = bb[q][z] - val;
        a.out[gcol[q] + m2 * gz] = val;
      }
    }
  }
};

}  // namespace pmg

// the operator apply that marches in z
#include "march.h"

// h-transfers and the coarse solve
#include "transfer.h"
