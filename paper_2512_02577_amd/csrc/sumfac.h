// Sum-factorized 1D contractions on small tensors held in LDS.
//
// A tensor of extents (E0, E1, E2) is stored x fastest.  A contraction along axis AX
// replaces extent E_AX = NIN by NOUT: out(.., o, ..) = sum_i Mat[o][i] in(.., i, ..).
// Each thread owns whole pencils (all NIN inputs of one line), loads them into
// registers once and produces every output of the line, so one LDS read feeds up to
// 2*NOUT fused multiply-adds.  Matrices are row-major NOUT x NIN tables in global memory
// with wave-uniform addresses (read through the scalar cache) and a compile-time
// sparsity pattern: row o touches columns [Pat::lo(o), Pat::hi(o)) only.
//
// The bodies are __host__ __device__: on the device tid/NT are the workgroup's threads;
// on the host the same code runs for index, bounds and race checks, either sequentially
// (NT = 1) or with one host thread per lane (a HostTeam, whose barrier stands in for the
// workgroup barrier).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define PMG_HD __host__ __device__
#define PMG_INLINE __host__ __device__ inline __attribute__((always_inline))
#else
#define PMG_HD
#define PMG_INLINE inline
#endif

#if defined(__HIP_DEVICE_COMPILE__)
#define PMG_SYNC() __syncthreads()
// Operator tables are read through the constant address space: wave-uniform addresses
// then become scalar loads into SGPRs instead of per-lane vector loads.
#define PMG_CONST_AS __attribute__((address_space(4)))
#else
namespace pmg {
// Host runs with one thread per lane register the team of the calling thread here; the
// workgroup barrier and the workgroup sum then go through it.  Without a team (NT = 1)
// the barrier is a no-op.
struct HostTeam {
  virtual ~HostTeam() = default;
  virtual void sync() = 0;
  virtual double sum(int tid, double v) = 0;  // every lane gets the sum in lane order
};
inline thread_local HostTeam *host_team = nullptr;
inline void host_sync() {
  if (host_team) host_team->sync();
}
}  // namespace pmg
#define PMG_SYNC() ::pmg::host_sync()
#define PMG_CONST_AS
#endif

namespace pmg {

template <typename T>
using cptr = const PMG_CONST_AS T *;

template <typename T>
PMG_INLINE cptr<T> as_const(const T *p) {
  return (cptr<T>)p;
}

// The same table pointer, as a value the compiler cannot carry over from an earlier pencil
// of the same loop: the matrix entries of each pencil are then loaded where they are used
// (scalar-cache hits) instead of being hoisted out of the pencil loop, where the entries
// of a 1D matrix outnumber the scalar registers and spill into vector-register lanes.
template <typename T>
PMG_INLINE cptr<T> per_pencil(cptr<T> p) {
#if defined(__HIP_DEVICE_COMPILE__)
  // the tables are the same on every lane: read the address from the first lane (a no-op
  // where it is already scalar) and pass it through an empty scalar asm operand
  const unsigned long long v = (unsigned long long)p;
  unsigned long long w = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(v >> 32)) << 32) |
                         (unsigned)__builtin_amdgcn_readfirstlane((unsigned)v);
  asm volatile("" : "+s"(w));
  return (cptr<T>)w;
#else
  return p;
#endif
}

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// ---- gathers from global memory ----------------------------------------------------------
// Two per-lane strided streams, e = tid, tid + NT, ... < C1 (then < C2), read from global
// memory and stored (to LDS or registers).  A rolled loop that stores each value right after
// its load waits for every load in turn; here the loads of up to G slots (both streams
// together) are issued before the first is consumed, so a lane waits about once per group.
// ld1/ld2 are called for every slot, with e clamped into range on the lanes past the end,
// so they must be branch-free loads valid for every e < C (select, do not skip); st1/st2
// run only for e < C.
template <int C1, int C2, int NT, int G, typename T, class L1, class S1, class L2, class S2>
PMG_INLINE void lane_gather2(int tid, L1 &&ld1, S1 &&st1, L2 &&ld2, S2 &&st2) {
  constexpr int R1 = (C1 + NT - 1) / NT, R2 = (C2 + NT - 1) / NT, R = R1 + R2;
  constexpr int GG = R < G ? R : G;
#pragma unroll
  for (int j0 = 0; j0 < R; j0 += GG) {
    T v[GG];
#pragma unroll
    for (int k = 0; k < GG; ++k) {
      const int j = j0 + k;
      if (j < R1) {
        const int e = tid + j * NT;
        v[k] = ld1(e < C1 ? e : C1 - 1);
      } else if (j < R) {
        const int e = tid + (j - R1) * NT;
        v[k] = ld2(e < C2 ? e : C2 - 1);
      }
    }
#if defined(__HIP_DEVICE_COMPILE__)
    // an empty asm that takes every value keeps the compiler from sinking a load into the
    // conditional store of its slot (which would wait for it there, alone)
#pragma unroll
    for (int k = 0; k < GG; ++k) asm volatile("" : "+v"(v[k]));
#endif
#pragma unroll
    for (int k = 0; k < GG; ++k) {
      const int j = j0 + k;
      if (j < R1) {
        const int e = tid + j * NT;
        if (e < C1) st1(e, v[k]);
      } else if (j < R) {
        const int e = tid + (j - R1) * NT;
        if (e < C2) st2(e, v[k]);
      }
    }
  }
}

template <int C, int NT, int G, typename T, class L, class S>
PMG_INLINE void lane_gather(int tid, L &&ld, S &&st) {
  lane_gather2<C, 0, NT, G, T>(tid, ld, st, [](int) { return T(0); }, [](int, T) {});
}

// ---- sparsity patterns of the 1D matrices ---------------------------------------------
// Patch interior matrix of degree Q: rows/cols are the 2Q-1 interior nodes of two cells.
template <int Q>
struct PatInterior {
  static constexpr int nout = 2 * Q - 1, nin = 2 * Q - 1;
  PMG_HD static constexpr int lo(int o) { return (o + 1 > Q) ? Q - 1 : 0; }
  PMG_HD static constexpr int hi(int o) { return (o + 1 < Q) ? Q : 2 * Q - 1; }
};
// Patch residual of degree P: interior rows (2P-1), closure columns (2P+1).
template <int P>
struct PatResidual {
  static constexpr int nout = 2 * P - 1, nin = 2 * P + 1;
  PMG_HD static constexpr int lo(int o) { return (o + 1 > P) ? P : 0; }
  PMG_HD static constexpr int hi(int o) { return (o + 1 < P) ? P + 1 : 2 * P + 1; }
};
// Embedding of degree QC into degree QF on a patch: fine interior rows, coarse interior cols.
template <int QF, int QC>
struct PatProlong {
  static constexpr int nout = 2 * QF - 1, nin = 2 * QC - 1;
  PMG_HD static constexpr int lo(int o) { return (o + 1 >= QF) ? QC - 1 : 0; }
  PMG_HD static constexpr int hi(int o) { return (o + 1 <= QF) ? QC : 2 * QC - 1; }
};
// Its transpose: coarse interior rows, fine interior cols.
template <int QF, int QC>
struct PatRestrict {
  static constexpr int nout = 2 * QC - 1, nin = 2 * QF - 1;
  PMG_HD static constexpr int lo(int o) { return (o + 1 > QC) ? QF - 1 : 0; }
  PMG_HD static constexpr int hi(int o) { return (o + 1 < QC) ? QF : 2 * QF - 1; }
};
// Apply tile of TC cells of degree P: output nodes P*c0 + o (o < P*TC), input nodes
// P*(c0-1) + i (i <= P*(TC+1)); row o touches the cells containing its node.
template <int P, int TC>
struct PatTile {
  static constexpr int nout = P * TC, nin = P * (TC + 1) + 1;
  PMG_HD static constexpr int lo(int o) { return (o % P == 0) ? P * (o / P) : P * (o / P + 1); }
  PMG_HD static constexpr int hi(int o) { return P * (o / P + 1) + P + 1; }
};

// A dense NO x NI matrix (every row touches every column).
template <int NO, int NI>
struct PatDense {
  static constexpr int nout = NO, nin = NI;
  PMG_HD static constexpr int lo(int) { return 0; }
  PMG_HD static constexpr int hi(int) { return NI; }
};

// ---- one output of a 1D contraction on a register pencil ------------------------------
// Row o of a matrix with sparsity Pat as one FMA chain seeded with its first product: an
// accumulator started at 0 costs one more instruction (0 + x is not folded away under IEEE
// signed zeros), and "acc += K a + M b" would round K a + M b first (mul, fma, add per
// term) instead of chaining two FMAs.
template <class Pat, typename T, class MP>
PMG_INLINE T row1(const MP &M, int o, const T *v) {
  const int l = Pat::lo(o), h = Pat::hi(o);
  if (h <= l) return T(0);
  T acc = M[o * Pat::nin + l] * v[l];
#pragma unroll
  for (int i = 0; i < Pat::nin; ++i)
    if (i > l && i < h) acc += M[o * Pat::nin + i] * v[i];
  return acc;
}

// Row o of K va + M vb (same pattern) as one FMA chain
template <class Pat, typename T, class MP>
PMG_INLINE T row2(const MP &K, const MP &M, int o, const T *va, const T *vb) {
  const int l = Pat::lo(o), h = Pat::hi(o);
  if (h <= l) return T(0);
  T acc = K[o * Pat::nin + l] * va[l];
  acc += M[o * Pat::nin + l] * vb[l];
#pragma unroll
  for (int i = 0; i < Pat::nin; ++i)
    if (i > l && i < h) {
      acc += K[o * Pat::nin + i] * va[i];
      acc += M[o * Pat::nin + i] * vb[i];
    }
  return acc;
}

// ---- axis bookkeeping -----------------------------------------------------------------
template <int AX, int E0, int E1, int E2, int NOUT>
struct Axis {
  static constexpr int NIN = AX == 0 ? E0 : (AX == 1 ? E1 : E2);
  static constexpr int NPEN = E0 * E1 * E2 / NIN;
  static constexpr int IS = AX == 0 ? 1 : (AX == 1 ? E0 : E0 * E1);  // input stride on AX
  static constexpr int OS = AX == 0 ? 1 : (AX == 1 ? E0 : E0 * E1);  // output stride on AX
  PMG_INLINE static void base(int pen, int &ib, int &ob) {
    if (AX == 0) {
      ib = pen * E0;
      ob = pen * NOUT;
    } else if (AX == 1) {
      int i = pen % E0, k = pen / E0;
      ib = i + E0 * E1 * k;
      ob = i + E0 * NOUT * k;
    } else {
      ib = pen;
      ob = pen;
    }
  }
};

// oa = A in, ob = B in  (same pattern)
template <int AX, int E0, int E1, int E2, class Pat, int NT, typename T>
PMG_INLINE void contract2(int tid, const T *in, T *oa, const T *A_, T *ob, const T *B_) {
  using X = Axis<AX, E0, E1, E2, Pat::nout>;
  const cptr<T> A0 = as_const(A_), B0 = as_const(B_);
  static_assert(X::NIN == Pat::nin, "extent mismatch");
  for (int pen = tid; pen < X::NPEN; pen += NT) {
    const cptr<T> A = per_pencil(A0), B = per_pencil(B0);
    int ib, obs;
    X::base(pen, ib, obs);
    T v[Pat::nin];
#pragma unroll
    for (int i = 0; i < Pat::nin; ++i) v[i] = in[ib + i * X::IS];
#pragma unroll
    for (int o = 0; o < Pat::nout; ++o) {
      oa[obs + o * X::OS] = row1<Pat>(A, o, v);
      ob[obs + o * X::OS] = row1<Pat>(B, o, v);
    }
  }
}

// oc = M ia, og = K ia + M ib
template <int AX, int E0, int E1, int E2, class Pat, int NT, typename T>
PMG_INLINE void contract_pair(int tid, const T *ia, const T *ib_, T *oc, T *og, const T *M_, const T *K_) {
  using X = Axis<AX, E0, E1, E2, Pat::nout>;
  const cptr<T> M0 = as_const(M_), K0 = as_const(K_);
  static_assert(X::NIN == Pat::nin, "extent mismatch");
  for (int pen = tid; pen < X::NPEN; pen += NT) {
    const cptr<T> M = per_pencil(M0), K = per_pencil(K0);
    int ib, obs;
    X::base(pen, ib, obs);
    T va[Pat::nin], vb[Pat::nin];
#pragma unroll
    for (int i = 0; i < Pat::nin; ++i) {
      va[i] = ia[ib + i * X::IS];
      vb[i] = ib_[ib + i * X::IS];
    }
#pragma unroll
    for (int o = 0; o < Pat::nout; ++o) {
      oc[obs + o * X::OS] = row1<Pat>(M, o, va);
      og[obs + o * X::OS] = row2<Pat>(K, M, o, va, vb);
    }
  }
}

// out = base - s (K ia + M ib)   (base != nullptr), or out = s (K ia + M ib)
template <int AX, int E0, int E1, int E2, class Pat, int NT, typename T>
PMG_INLINE void contract_final(int tid, const T *ia, const T *ib_, T *out, const T *base, T s, const T *K_,
                               const T *M_) {
  using X = Axis<AX, E0, E1, E2, Pat::nout>;
  const cptr<T> K0 = as_const(K_), M0 = as_const(M_);
  static_assert(X::NIN == Pat::nin, "extent mismatch");
  for (int pen = tid; pen < X::NPEN; pen += NT) {
    const cptr<T> K = per_pencil(K0), M = per_pencil(M0);
    int ib, obs;
    X::base(pen, ib, obs);
    T va[Pat::nin], vb[Pat::nin];
#pragma unroll
    for (int i = 0; i < Pat::nin; ++i) {
      va[i] = ia[ib + i * X::IS];
      vb[i] = ib_[ib + i * X::IS];
    }
#pragma unroll
    for (int o = 0; o < Pat::nout; ++o) {
      const T acc = row2<Pat>(K, M, o, va, vb);
      const int oi = obs + o * X::OS;
      out[oi] = base ? base[oi] - s * acc : s * acc;
    }
  }
}

// out = Mat in  (ADD: out += Mat in)
template <int AX, int E0, int E1, int E2, class Pat, int NT, bool ADD, typename T>
PMG_INLINE void contract1(int tid, const T *in, T *out, const T *Mat_) {
  using X = Axis<AX, E0, E1, E2, Pat::nout>;
  const cptr<T> Mat0 = as_const(Mat_);
  static_assert(X::NIN == Pat::nin, "extent mismatch");
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
      if (ADD)
        out[oi] += acc;
      else
        out[oi] = acc;
    }
  }
}

// ---- whole-tensor Laplacian pieces ----------------------------------------------------
// out = base - s * (sum_k K_k (x) M_others) in,  in: (N,N,N) or (N,N) through a pattern
// Pat (N = Pat::nin -> n = Pat::nout per axis).  Scratch: ab (2 n N^(d-1)), cg (2 n^2 N).
// in and cg may alias (in is dead after the first stage).
template <int DIM, class Pat, int NT, typename T>
PMG_INLINE void laplace_sf(int tid, const T *in, T *out, const T *base, T s, const T *K, const T *M,
                           T *ab, T *cg) {
  constexpr int N = Pat::nin, n = Pat::nout;
  if constexpr (DIM == 3) {
    constexpr int SA = n * N * N, SC = n * n * N;
    contract2<0, N, N, N, Pat, NT>(tid, in, ab, M, ab + SA, K);  // A = Mx u, B = Kx u
    PMG_SYNC();
    contract_pair<1, n, N, N, Pat, NT>(tid, ab, ab + SA, cg, cg + SC, M, K);  // C = My A, G = Ky A + My B
    PMG_SYNC();
    contract_final<2, n, n, N, Pat, NT>(tid, cg, cg + SC, out, base, s, K, M);  // Kz C + Mz G
  } else {
    constexpr int SA = n * N;
    contract2<0, N, N, 1, Pat, NT>(tid, in, ab, M, ab + SA, K);
    PMG_SYNC();
    contract_final<1, n, N, 1, Pat, NT>(tid, ab, ab + SA, out, base, s, K, M);  // Ky A + My B
  }
}

constexpr int lap_ab(int dim, int N, int n) { return dim == 3 ? 2 * n * N * N : 2 * n * N; }
constexpr int lap_cg(int dim, int N, int n) { return dim == 3 ? 2 * n * n * N : 0; }
template <int DIM, int N, int n>
struct LapScratch {
  static constexpr int ab = lap_ab(DIM, N, n);
  static constexpr int cg = lap_cg(DIM, N, n);
};

// out (= or +=) Kronecker product of the 1D matrix Mat (pattern Pat) in every direction.
// Scratch t1 (NOUT NIN^(d-1)), t2 (NOUT^2 NIN) for 3D.
template <int DIM, class Pat, int NT, bool ADD, typename T>
PMG_INLINE void kron_all(int tid, const T *in, T *out, const T *Mat, T *t1, T *t2) {
  constexpr int I = Pat::nin, O = Pat::nout;
  if constexpr (DIM == 3) {
    contract1<0, I, I, I, Pat, NT, false>(tid, in, t1, Mat);
    PMG_SYNC();
    contract1<1, O, I, I, Pat, NT, false>(tid, t1, t2, Mat);
    PMG_SYNC();
    contract1<2, O, O, I, Pat, NT, ADD>(tid, t2, out, Mat);
  } else {
    contract1<0, I, I, 1, Pat, NT, false>(tid, in, t1, Mat);
    PMG_SYNC();
    contract1<1, O, I, 1, Pat, NT, ADD>(tid, t1, out, Mat);
  }
}

constexpr int kron_t1(int dim, int I, int O) { return dim == 3 ? O * I * I : O * I; }
constexpr int kron_t2(int dim, int I, int O) { return dim == 3 ? O * O * I : 0; }

// ---- strided pencils (contractions that may run in place) --------------------------------
// A tensor of logical extents (E0, E1, E2) stored with strides (1, S1, S2).  A contraction
// along AX reads each pencil into registers and writes its NOUT <= NIN outputs to the
// pencil positions 0..NOUT-1 of the output layout; since a pencil is read completely by
// the lane that owns it before that lane writes, and pencils of one axis are disjoint,
// the output may be the input buffer itself (same layout): no barrier between read and
// write, and no separate stage buffer.
template <int S1_, int S2_>
struct Lay {
  static constexpr int S1 = S1_, S2 = S2_;
};
template <int E0, int E1>
using Dense = Lay<E0, E0 * E1>;  // compact layout of extents (E0, E1, *)

template <int AX, int E0, int E1, int E2>
struct Pen {
  static constexpr int NIN = AX == 0 ? E0 : (AX == 1 ? E1 : E2);
  static constexpr int NA = AX == 0 ? E1 : E0;  // extent of the first other axis
  static constexpr int NB = AX == 2 ? E1 : E2;  // extent of the second other axis
  static constexpr int NPEN = NA * NB;
  template <class L>
  PMG_INLINE static int base(int pen) {
    const int a = pen % NA, b = pen / NA;
    return AX == 0 ? a * L::S1 + b * L::S2 : (AX == 1 ? a + b * L::S2 : a + b * L::S1);
  }
  template <class L>
  static constexpr int step() {
    return AX == 0 ? 1 : (AX == 1 ? L::S1 : L::S2);
  }
};

// Work split of one contraction stage.  When the workgroup has more waves than the
// stage has pencils to fill, the waves are grouped into `parts` (PW waves each, enough for
// all pencils) and part k computes the outputs [lo(k), hi(k)) of every pencil: each wave
// reads whole pencils but does a share of the multiply-adds, which shortens the stage
// (the latency of a patch is a chain of such stages).  The part is wave-uniform, so the
// output range is a compile-time constant in every branch and the matrix entries stay
// scalar operands.  A split stage that writes in place (INPL) has a barrier between
// reading the pencils and writing them, since another part may still read what one part
// overwrites.  On the host (NT = 1) there is one part.
template <int NPEN, int NOUT, int NT>
struct WSplit {
  static constexpr int NW = NT / 64;
  static constexpr int PW = (NPEN + 63) / 64;
  static constexpr int P0 = NW >= 2 * PW ? NW / PW : 1;
  static constexpr int parts = P0 < NOUT ? P0 : NOUT;
  static constexpr int lo(int k) { return k * NOUT / parts; }
  static constexpr int hi(int k) { return (k + 1) * NOUT / parts; }
  // f.load(pen, regs); f.template store<lo(k), hi(k)>(pen, regs) for this lane's pencils
  template <bool INPL, class F>
  PMG_INLINE static void each(int tid, const F &f) {
    typename F::Regs r;
    if constexpr (parts == 1) {
      for (int pen = tid; pen < NPEN; pen += NT) {
        f.load(pen, r);
        f.template store<0, NOUT>(pen, r);
      }
    } else {
      // part is the same on every lane of a wave (64 PW lanes per part); saying so makes
      // the part branches scalar, so each keeps its matrix entries as scalar operands
#if defined(__HIP_DEVICE_COMPILE__)
      const int part = __builtin_amdgcn_readfirstlane(tid / (64 * PW));
#else
      const int part = tid / (64 * PW);
#endif
      const int pen = tid % (64 * PW);
      const bool act = part < parts && pen < NPEN;
      if (act) f.load(pen, r);
      if constexpr (INPL) PMG_SYNC();
      if (act) dispatch<0>(part, pen, r, f);
    }
  }
  template <int K, class F>
  PMG_INLINE static void dispatch(int part, int pen, const typename F::Regs &r, const F &f) {
    if constexpr (K < parts) {
      if (part == K)
        f.template store<lo(K), hi(K)>(pen, r);
      else
        dispatch<K + 1>(part, pen, r, f);
    }
  }
};

// Pencil functors of the contractions below: load a pencil into registers, then produce
// the outputs [O0, O1) of it.
template <int AX, int E0, int E1, int E2, class Pat, class LI, class LA, class LB, typename T>
struct FC2 {  // oa = A in, ob = B in
  using X = Pen<AX, E0, E1, E2>;
  const T *in;
  T *oa, *ob;
  cptr<T> A, B;
  struct Regs {
    T v[Pat::nin];
  };
  PMG_INLINE void load(int pen, Regs &r) const {
    const int ib = X::template base<LI>(pen);
#pragma unroll
    for (int i = 0; i < Pat::nin; ++i) r.v[i] = in[ib + i * X::template step<LI>()];
  }
  template <int O0, int O1>
  PMG_INLINE void store(int pen, const Regs &r) const {
    const int oab = X::template base<LA>(pen), obb = X::template base<LB>(pen);
    const cptr<T> Ap = per_pencil(A), Bp = per_pencil(B);
#pragma unroll
    for (int o = O0; o < O1; ++o) {
      oa[oab + o * X::template step<LA>()] = row1<Pat>(Ap, o, r.v);
      ob[obb + o * X::template step<LB>()] = row1<Pat>(Bp, o, r.v);
    }
  }
};

template <int AX, int E0, int E1, int E2, class Pat, class LA, class LB, typename T>
struct FCPair {  // ia <- M ia, ib <- K ia + M ib
  using X = Pen<AX, E0, E1, E2>;
  T *ia, *ib;
  cptr<T> M, K;
  struct Regs {
    T va[Pat::nin], vb[Pat::nin];
  };
  PMG_INLINE void load(int pen, Regs &r) const {
    const int ab = X::template base<LA>(pen), bb = X::template base<LB>(pen);
#pragma unroll
    for (int i = 0; i < Pat::nin; ++i) {
      r.va[i] = ia[ab + i * X::template step<LA>()];
      r.vb[i] = ib[bb + i * X::template step<LB>()];
    }
  }
  template <int O0, int O1>
  PMG_INLINE void store(int pen, const Regs &r) const {
    const int ab = X::template base<LA>(pen), bb = X::template base<LB>(pen);
    const cptr<T> Mp = per_pencil(M), Kp = per_pencil(K);
#pragma unroll
    for (int o = O0; o < O1; ++o) {
      ia[ab + o * X::template step<LA>()] = row1<Pat>(Mp, o, r.va);
      ib[bb + o * X::template step<LB>()] = row2<Pat>(Kp, Mp, o, r.va, r.vb);
    }
  }
};

template <int AX, int E0, int E1, int E2, class Pat, class LA, class LB, class LO, typename T>
struct FCFinal {  // out = base - s (K ia + M ib)
  using X = Pen<AX, E0, E1, E2>;
  const T *ia, *ib;
  T *out;
  const T *base;
  T s;
  cptr<T> K, M;
  struct Regs {
    T va[Pat::nin], vb[Pat::nin];
  };
  PMG_INLINE void load(int pen, Regs &r) const {
    const int ab = X::template base<LA>(pen), bb = X::template base<LB>(pen);
#pragma unroll
    for (int i = 0; i < Pat::nin; ++i) {
      r.va[i] = ia[ab + i * X::template step<LA>()];
      r.vb[i] = ib[bb + i * X::template step<LB>()];
    }
  }
  template <int O0, int O1>
  PMG_INLINE void store(int pen, const Regs &r) const {
    const int ob = X::template base<LO>(pen);
    const cptr<T> Kp = per_pencil(K), Mp = per_pencil(M);
#pragma unroll
    for (int o = O0; o < O1; ++o) {
      const T acc = row2<Pat>(Kp, Mp, o, r.va, r.vb);
      const int oi = ob + o * X::template step<LO>();
      out[oi] = base[oi] - s * acc;
    }
  }
};

template <int AX, int E0, int E1, int E2, class Pat, bool ADD, class LI, class LO, typename T>
struct FC1 {  // out (=|+=) Mat in
  using X = Pen<AX, E0, E1, E2>;
  const T *in;
  T *out;
  cptr<T> Mat;
  struct Regs {
    T v[Pat::nin];
  };
  PMG_INLINE void load(int pen, Regs &r) const {
    const int ib = X::template base<LI>(pen);
#pragma unroll
    for (int i = 0; i < Pat::nin; ++i) r.v[i] = in[ib + i * X::template step<LI>()];
  }
  template <int O0, int O1>
  PMG_INLINE void store(int pen, const Regs &r) const {
    const int ob = X::template base<LO>(pen);
    const cptr<T> Mp = per_pencil(Mat);
#pragma unroll
    for (int o = O0; o < O1; ++o) {
      const T acc = row1<Pat>(Mp, o, r.v);
      const int oi = ob + o * X::template step<LO>();
      if (ADD)
        out[oi] += acc;
      else
        out[oi] = acc;
    }
  }
};

// oa = A in (layout LA), ob = B in (layout LB); INPL: oa is in (LA = LI)
template <int AX, int E0, int E1, int E2, class Pat, int NT, class LI, class LA, class LB, bool INPL = false,
          typename T>
PMG_INLINE void scontract2(int tid, const T *in, T *oa, const T *A_, T *ob, const T *B_) {
  using F = FC2<AX, E0, E1, E2, Pat, LI, LA, LB, T>;
  static_assert(F::X::NIN == Pat::nin, "extent mismatch");
  WSplit<F::X::NPEN, Pat::nout, NT>::template each<INPL>(tid, F{in, oa, ob, as_const(A_), as_const(B_)});
}

// ia <- M ia, ib <- K ia + M ib, in place (layouts LA, LB)
template <int AX, int E0, int E1, int E2, class Pat, int NT, class LA, class LB, typename T>
PMG_INLINE void scontract_pair(int tid, T *ia, T *ib, const T *M_, const T *K_) {
  using F = FCPair<AX, E0, E1, E2, Pat, LA, LB, T>;
  static_assert(F::X::NIN == Pat::nin, "extent mismatch");
  WSplit<F::X::NPEN, Pat::nout, NT>::template each<true>(tid, F{ia, ib, as_const(M_), as_const(K_)});
}

// out = base - s (K ia + M ib) (base may be out), out in layout LO; INPL: out is ia
template <int AX, int E0, int E1, int E2, class Pat, int NT, class LA, class LB, class LO, bool INPL = false,
          typename T>
PMG_INLINE void scontract_final(int tid, const T *ia, const T *ib, T *out, const T *base, T s, const T *K_,
                                const T *M_) {
  using F = FCFinal<AX, E0, E1, E2, Pat, LA, LB, LO, T>;
  static_assert(F::X::NIN == Pat::nin, "extent mismatch");
  WSplit<F::X::NPEN, Pat::nout, NT>::template each<INPL>(tid, F{ia, ib, out, base, s, as_const(K_), as_const(M_)});
}

// out = Mat in (ADD: out += Mat in); INPL: out is in (LO = LI, NOUT <= NIN)
template <int AX, int E0, int E1, int E2, class Pat, int NT, bool ADD, class LI, class LO, bool INPL = false,
          typename T>
PMG_INLINE void scontract1(int tid, const T *in, T *out, const T *Mat_) {
  using F = FC1<AX, E0, E1, E2, Pat, ADD, LI, LO, T>;
  static_assert(F::X::NIN == Pat::nin, "extent mismatch");
  WSplit<F::X::NPEN, Pat::nout, NT>::template each<INPL>(tid, F{in, out, as_const(Mat_)});
}

template <int AX, int E0, int E1, int E2, class Pat, class LI, class LO, typename T>
struct FCSub {  // out = base - Mat in
  using X = Pen<AX, E0, E1, E2>;
  const T *in;
  T *out;
  const T *base;
  cptr<T> Mat;
  struct Regs {
    T v[Pat::nin];
  };
  PMG_INLINE void load(int pen, Regs &r) const {
    const int ib = X::template base<LI>(pen);
#pragma unroll
    for (int i = 0; i < Pat::nin; ++i) r.v[i] = in[ib + i * X::template step<LI>()];
  }
  template <int O0, int O1>
  PMG_INLINE void store(int pen, const Regs &r) const {
    const int ob = X::template base<LO>(pen);
    const cptr<T> Mp = per_pencil(Mat);
#pragma unroll
    for (int o = O0; o < O1; ++o) {
      const T acc = row1<Pat>(Mp, o, r.v);
      const int oi = ob + o * X::template step<LO>();
      out[oi] = base[oi] - acc;
    }
  }
};

// Compact tensors: the layout of the input (E0, E1, E2) and of the output along AX.
template <int AX, int E0, int E1, int NOUT>
using DenseOut = Dense<AX == 0 ? NOUT : E0, AX == 1 ? NOUT : E1>;

// out (=|+=) Mat in on compact tensors (out-of-place, or in place along AX with INPL and
// NOUT = NIN), split over waves like the strided contractions
template <int AX, int E0, int E1, int E2, class Pat, int NT, bool ADD, bool INPL = false, typename T>
PMG_INLINE void dcontract1(int tid, const T *in, T *out, const T *Mat) {
  scontract1<AX, E0, E1, E2, Pat, NT, ADD, Dense<E0, E1>, DenseOut<AX, E0, E1, Pat::nout>, INPL>(tid, in, out, Mat);
}

// out = base - Mat in on compact tensors (out-of-place)
template <int AX, int E0, int E1, int E2, class Pat, int NT, typename T>
PMG_INLINE void dcontract_sub(int tid, const T *in, T *out, const T *base, const T *Mat_) {
  using F = FCSub<AX, E0, E1, E2, Pat, Dense<E0, E1>, DenseOut<AX, E0, E1, Pat::nout>, T>;
  static_assert(F::X::NIN == Pat::nin, "extent mismatch");
  WSplit<F::X::NPEN, Pat::nout, NT>::template each<false>(tid, F{in, out, base, as_const(Mat_)});
}

// Sum over the workgroup of one value per lane; every lane gets the total.  red: NT/64
// (at least 1) elements of LDS scratch.  On the host the value itself (NT = 1) or the
// team's sum.
template <int NT, typename T>
PMG_INLINE T block_sum(int tid, T v, T *red) {
#if defined(__HIP_DEVICE_COMPILE__)
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  constexpr int NW = NT / 64 > 0 ? NT / 64 : 1;
  if (NW == 1) return v;
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += red[w];
  __syncthreads();
  return s;
#else
  (void)red;
  if constexpr (NT == 1) {
    (void)tid;
    return v;
  } else {
    return (T)host_team->sum(tid, (double)v);
  }
#endif
}

}  // namespace pmg
