// Operator apply on the Cartesian mesh that marches through the mesh in z (3D only).
//
// v = A u with A = c sum_d K_d (x) M_others (Sec. 3.1, Eq. 3: the cell matrices of the
// uniform mesh factor into 1D stiffness and mass matrices), or its residual form b - A u, or
// the mass matrix v = c M (x) M (x) M u.  Rows and columns of the Dirichlet boundary nodes are
// those of the identity (zero for the mass matrix).
//
// A workgroup owns an xy tile of TX x TX cells and a segment of cell layers in z, and walks
// up the segment one cell layer at a time.  Per layer, the z contraction comes first and runs
// in registers: every lane owns whole z columns of the tile's input (TX + 2 cells wide in x
// and y, the owned cells and one halo cell on each side) and keeps a window of the 2P + 1
// planes of the cells below and above the layer's owned planes; the P new planes of the next
// layer are loaded while the current one is computed, and the window moves up by P planes.
// The y and x contractions then run in LDS on the layer's P planes, one lane per cell
// segment (the P owned nodes of one cell along a line, read from the 2P + 1 nodes of the two
// cells that touch them).  The z halo costs P + 1 plane loads at the start of a segment and
// no arithmetic; the xy halo is re-read by the neighbouring tiles (from L2).
//
// Order of the contractions (any order gives the same operator): Zm = Mz u, Zk = Kz u;
// Ym = My Zm, Yg = Ky Zm + My Zk; v = c (Kx Ym + Mx Yg).  Mass: Zm, Ym = My Zm, v = c Mx Ym.
// A y or x unit reads its first field, starts the FMA chains of its outputs, then reads the
// second field into the same registers and continues them: half the input registers of
// reading both at once (the register count, not the LDS, sets the occupancy from p = 6 on).
#pragma once

namespace pmg {

// Rows of the owned nodes of one cell along a line: node o (o = 0 is the vertex shared with
// the cell below) reads the 2P + 1 nodes t of the cell below and its own, taps t >= P only
// for o > 0.  On the uniform mesh every entry is one of the 1D cell matrix C ((P+1) x (P+1),
// symmetric, and unchanged under reversing the cell: C[a][b] = C[P-a][P-b]) except the
// vertex's own, C[P][P] + C[0][0].  The taps are read from the first P rows of the apply
// tile tables (row stride TS) at one canonical position per class of equal entries, so a
// kernel needs about (P+1)(P+3)/4 scalar registers of entries per matrix, not P(P+2).
template <int P, int TS>
struct CellRows {
  static constexpr int lo(int o) { return o == 0 ? 0 : P; }
  // table position of the cell entry C[a][b] (a, b not both 0 or both P): row 0 holds
  // C[P][b] at b and C[0][b] at P + b, row a in 1..P-1 holds C[a][b] at P + b
  static constexpr int at(int a, int b) { return a == 0 ? P + b : (a == P ? b : a * TS + P + b); }
  static constexpr int canon(int a, int b) {
    int ra = a, rb = b;
    const int ca[3] = {b, P - a, P - b}, cb[3] = {a, P - b, P - a};
    for (int k = 0; k < 3; ++k)
      if (ca[k] < ra || (ca[k] == ra && cb[k] < rb)) ra = ca[k], rb = cb[k];
    return at(ra, rb);
  }
  static constexpr int idx(int o, int t) {
    if (o == 0) return t == P ? P : (t < P ? canon(P, t) : canon(0, t - P));
    return canon(o, t - P);
  }
};

// Row o of M v as one FMA chain
template <class R, int P, typename T, class MP>
PMG_INLINE T cell_row1(const MP &M, int o, const T *v) {
  const int l = R::lo(o);
  T acc = M[R::idx(o, l)] * v[l];
#pragma unroll
  for (int t = 0; t <= 2 * P; ++t)
    if (t > l) acc += M[R::idx(o, t)] * v[t];
  return acc;
}
// acc + row o of M v, continuing acc's FMA chain
template <class R, int P, typename T, class MP>
PMG_INLINE T cell_row_add(const MP &M, int o, const T *v, T acc) {
  const int l = R::lo(o);
#pragma unroll
  for (int t = 0; t <= 2 * P; ++t)
    if (t >= l) acc += M[R::idx(o, t)] * v[t];
  return acc;
}

// The outputs of one cell layer (its P planes), written through a buffer resource: a store
// at an offset past the end is dropped by the hardware, so the lanes without an output item
// store too, and no branch surrounds the stores.  (Around a branch the compiler's wait for
// the next layer's loads, which are older than the stores, would also wait for the stores.)
template <typename T>
struct LayerOut {
  static constexpr int kNone = 0x7fffffff;  // byte offset of "no output"
#if defined(__HIP_DEVICE_COMPILE__)
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  __amdgpu_buffer_rsrc_t r;
  PMG_INLINE LayerOut(T *base, int bytes) : r(__builtin_amdgcn_make_buffer_rsrc(base, (short)0, bytes, 0x00020000)) {}
  PMG_INLINE void put(int byte_off, T v) const {
    if constexpr (sizeof(T) == 8)
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, byte_off, 0, 0);
    else
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, byte_off, 0, 0);
  }
#else
  T *b;
  int n;
  LayerOut(T *base, int bytes) : b(base), n(bytes) {}
  void put(int byte_off, T v) const {
    if (byte_off >= 0 && byte_off < n) b[byte_off / (int)sizeof(T)] = v;
  }
#endif
};

// Largest mesh the marching apply takes: the byte offsets within one cell layer are ints.
template <typename T>
constexpr bool march_fits(int p, long m) {
  return (long)p * m * m * (long)sizeof(T) < (long)LayerOut<T>::kNone;
}

template <typename T, int NT, int P, int TX, int TY, int G, int TS, bool RESID, bool MASS>
struct MarchBody {
  static_assert(!(RESID && MASS), "the mass apply has no residual form");
  // input nodes (tile and halo) and owned nodes per direction, z columns
  static constexpr int NIX = P * (TX + 1) + 1, NIY = P * (TY + 1) + 1, NOX = P * TX, NOY = P * TY;
  static constexpr int NC = NIX * NIY;
  static constexpr int W = 2 * P + 1;            // z window: planes P(k-1) .. P(k+1) of layer k
  static constexpr int QZ = (NC + NT - 1) / NT;  // z columns per lane
  static constexpr int NF = MASS ? 1 : 2;        // fields after the z and y stages
  static constexpr int NG = (P + G - 1) / G;     // plane groups per layer (G planes each, the last fewer)
  static constexpr int SZ = G * NC, SY = G * NOY * NIX;
  static constexpr int OS = NOX + 1, SO = G * NOY * OS;  // staged outputs, rows padded by one
  static constexpr int NSX = NOX + 1, NSY = NOY + 1, NSS = NSX * NSY;
  static constexpr int QS = (NSS * G + NT - 1) / NT;  // store items per lane and group
  static constexpr int size = NF * SZ + NF * SY;
  static_assert(SO <= NF * SZ, "the staged outputs overlay the z-stage fields");
  using R = CellRows<P, TS>;

  PMG_INLINE static void run(int tid, int blk, T *lds, const ApplyArgs<T> &a) {
    const int t = xcd_remap(blk, a.n_tiles);
    const int mx = a.mt, my = a.mty;
    const int cx0 = TX * (t % mx), cy0 = TY * ((t / mx) % my), sg = t / (mx * my);
    const int n = a.n, m = P * n + 1;
    const size_t m2 = (size_t)m * m;
    const int k0 = a.zc * sg, k1 = k0 + a.zc < n ? k0 + a.zc : n;
    const T *__restrict__ u = a.u;
    T *zm = lds, *zk = lds + SZ, *ym = lds + NF * SZ, *yg = ym + SY, *ost = lds;
    const cptr<T> K0 = as_const(a.Kt), M0 = as_const(a.Mt);

    // ---- z columns of this lane: (i, j) of the NIX x NIY input nodes from P (cx0 - 1)
    int coff[QZ];
    bool cok[QZ];
#pragma unroll
    for (int q = 0; q < QZ; ++q) {
      int e = tid + q * NT;
      e = e < NC ? e : NC - 1;
      const int gx = P * (cx0 - 1) + e % NIX, gy = P * (cy0 - 1) + e / NIX;
      cok[q] = gx > 0 && gx < m - 1 && gy > 0 && gy < m - 1;
      const int cx = gx < 0 ? 0 : (gx > m - 1 ? m - 1 : gx), cy = gy < 0 ? 0 : (gy > m - 1 ? m - 1 : gy);
      coff[q] = cx + m * cy;
    }
    // node (column q, plane gz) as loaded: the address is clamped into the mesh; nodes outside
    // it or on its boundary are zeroed where the value enters the window (keep), not at the
    // load, so that a load in flight is not waited for until the window needs it
    auto raw = [&](int q, int gz) {
      const int cz = gz < 0 ? 0 : (gz > m - 1 ? m - 1 : gz);
      return u[coff[q] + m2 * cz];
    };
    auto keep = [&](int q, int gz) { return cok[q] && gz > 0 && gz < m - 1; };

    // ---- store items of this lane: (ox, oy, o) of (NOX + 1) x (NOY + 1) x G per plane
    // group; the extra row and column exist only where the tile ends at the upper mesh face
    // (there they are boundary nodes)
    const int bx = (cx0 + TX >= n ? m : P * (cx0 + TX)) - P * cx0;
    const int by = (cy0 + TY >= n ? m : P * (cy0 + TY)) - P * cy0;
    const bool edge = cx0 == 0 || cy0 == 0 || k0 == 0 || cx0 + TX >= n || cy0 + TY >= n;
    int soff[QS];
    bool sval[QS], sbxy[QS];
#pragma unroll
    for (int s = 0; s < QS; ++s) {
      const int e = tid + s * NT, ex = e % NSX, ey = (e / NSX) % NSY;
      sval[s] = e < NSS * G && ex < bx && ey < by;
      const int gx = P * cx0 + ex, gy = P * cy0 + ey;
      sbxy[s] = gx == 0 || gx == m - 1 || gy == 0 || gy == m - 1;
      soff[s] = sval[s] ? gx + m * gy : 0;
    }

    // ---- window of the first layer: planes P (k0 - 1) .. P (k0 + 1)
    T w[QZ][W];
#pragma unroll
    for (int q = 0; q < QZ; ++q)
#pragma unroll
      for (int tz = 0; tz < W; ++tz) {
        const int gz = P * (k0 - 1) + tz;
        const T x = raw(q, gz);
        w[q][tz] = keep(q, gz) ? x : T(0);
      }

    for (int k = k0; k < k1; ++k) {
      T pf[QZ][P];
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const int g0 = g * G;
        const int GG = P - g0 < G ? P - g0 : G;  // planes of this group
        // b, and u at boundary nodes, for this group's stores; the first group's are issued
        // before the prefetch below, so that its stores wait for these loads only
        T sb[QS], su[QS] = {};
        const size_t zoff = m2 * (size_t)(P * k + g0);
#pragma unroll
        for (int s = 0; s < QS; ++s) {
          const int o = (tid + s * NT) / NSS;
          const size_t gi = zoff + m2 * (size_t)(o < GG ? o : GG - 1) + soff[s];
          if constexpr (RESID) sb[s] = a.b[gi];
          if (!MASS && edge) su[s] = u[gi];
        }
        if (g == 0) {
          // the next layer's new planes, in flight during this layer and taken into the window
          // at its end (after the segment's last layer its top plane again: no branch, and no
          // new traffic); the window is carried from layer to layer, these registers are not
#pragma unroll
          for (int q = 0; q < QZ; ++q)
#pragma unroll
            for (int tz = 0; tz < P; ++tz) {
              const int gz = P * (k + 1) + 1 + tz;
              pf[q][tz] = raw(q, gz < P * k1 ? gz : P * k1);
            }
        }
        // z stage: Zm = Mz u, Zk = Kz u at the group's owned planes
#pragma unroll
        for (int q = 0; q < QZ; ++q) {
          const int e = tid + q * NT;
          if (NC % NT != 0 && e >= NC) continue;
#pragma unroll
          for (int o = 0; o < G; ++o) {
            if (o >= GG) continue;
            zm[o * NC + e] = cell_row1<R, P>(M0, g0 + o, w[q]);
            if constexpr (!MASS) zk[o * NC + e] = cell_row1<R, P>(K0, g0 + o, w[q]);
          }
        }
        PMG_SYNC();
        // y stage: one lane per (x node i, y cell cy, plane o)
        for (int v = tid; v < NIX * TY * GG; v += NT) {
          const int i = v % NIX, cy = (v / NIX) % TY, o = v / (NIX * TY);
          const int ib = o * NC + P * cy * NIX + i, ob = o * NOY * NIX + P * cy * NIX + i;
          T za[W], acc[MASS ? 1 : P];
#pragma unroll
          for (int tz = 0; tz < W; ++tz) za[tz] = zm[ib + tz * NIX];
#pragma unroll
          for (int oy = 0; oy < P; ++oy) {
            ym[ob + oy * NIX] = cell_row1<R, P>(M0, oy, za);
            if constexpr (!MASS) acc[oy] = cell_row1<R, P>(K0, oy, za);
          }
          if constexpr (!MASS) {
            // the second field after the first is dead: its registers take the window
#pragma unroll
            for (int tz = 0; tz < W; ++tz) za[tz] = zk[ib + tz * NIX];
#pragma unroll
            for (int oy = 0; oy < P; ++oy) yg[ob + oy * NIX] = cell_row_add<R, P>(M0, oy, za, acc[oy]);
          }
        }
        PMG_SYNC();
        // x stage: one lane per (y node jo, x cell cx, plane o); outputs staged over the z fields
        for (int v = tid; v < NOY * TX * GG; v += NT) {
          const int jo = v % NOY, cx = (v / NOY) % TX, o = v / (NOY * TX);
          const int ib = o * NOY * NIX + jo * NIX + P * cx;
          T ya[W], acc[P];
#pragma unroll
          for (int tz = 0; tz < W; ++tz) ya[tz] = ym[ib + tz];
#pragma unroll
          for (int ox = 0; ox < P; ++ox) acc[ox] = MASS ? cell_row1<R, P>(M0, ox, ya) : cell_row1<R, P>(K0, ox, ya);
          if constexpr (!MASS) {
#pragma unroll
            for (int tz = 0; tz < W; ++tz) ya[tz] = yg[ib + tz];
#pragma unroll
            for (int ox = 0; ox < P; ++ox) acc[ox] = cell_row_add<R, P>(M0, ox, ya, acc[ox]);
          }
#pragma unroll
          for (int ox = 0; ox < P; ++ox) ost[o * NOY * OS + jo * OS + P * cx + ox] = a.c * acc[ox];
        }
        PMG_SYNC();
        if (g == NG - 1) {
          // the window moves up one layer, before the last group's stores are issued: the
          // loads it waits for are then the oldest in flight
#pragma unroll
          for (int q = 0; q < QZ; ++q) {
#pragma unroll
            for (int tz = 0; tz <= P; ++tz) w[q][tz] = w[q][tz + P];
#pragma unroll
            for (int tz = 0; tz < P; ++tz) w[q][P + 1 + tz] = keep(q, P * (k + 1) + 1 + tz) ? pf[q][tz] : T(0);
          }
        }
        const LayerOut<T> lout(a.out + zoff, (int)((size_t)GG * m2 * sizeof(T)));
#pragma unroll
        for (int s = 0; s < QS; ++s) {
          const int e = tid + s * NT, ex = e % NSX, ey = (e / NSX) % NSY, e2 = e / NSS, o = e2 < GG ? e2 : GG - 1;
          const bool bnd = sbxy[s] || P * k + g0 + o == 0;  // no owned plane of a layer is the top face
          const int lx = ex < NOX ? ex : NOX - 1, ly = ey < NOY ? ey : NOY - 1;
          T val = ost[o * NOY * OS + ly * OS + lx];
          val = (ex < NOX && ey < NOY) ? val : T(0);  // the extra row and column: boundary nodes
          if (edge && bnd) val = MASS ? T(0) : su[s];
          if constexpr (RESID) val = sb[s] - val;
          const bool st = sval[s] && e2 < GG;
          lout.put(st ? (int)(((size_t)o * m2 + soff[s]) * sizeof(T)) : LayerOut<T>::kNone, val);
        }
        PMG_SYNC();
      }
    }
    if (k1 == n) {  // the top face of the mesh: boundary nodes only
      const size_t zoff = m2 * (size_t)(m - 1);
      for (int e = tid; e < NSS; e += NT) {
        const int ex = e % NSX, ey = e / NSX;
        if (ex >= bx || ey >= by) continue;
        const size_t g = zoff + (P * cx0 + ex) + (size_t)m * (P * cy0 + ey);
        T val = MASS ? T(0) : u[g];
        if constexpr (RESID) val = a.b[g] - val;
        a.out[g] = val;
      }
    }
  }
};

}  // namespace pmg
