// Layout of the table block of one problem: every 1D table of host_tables.h
// concatenated in one device buffer (each table padded to a multiple of 32 entries plus
// 32 more, so that scalar loads that round an address up stay inside the block), and the
// DevTabs pointers into it.  The library uploads this block; the CPU emulation of the
// kernel bodies binds the same layout to check it.
#pragma once

#include <cstddef>
#include <vector>

#include "bodies.h"
#include "host_tables.h"

namespace pmg {

template <typename T>
void bind_tabs(DevTabs<T> &d, const Tables &t, T *base, const std::vector<size_t> &off) {
  size_t k = 0;
  for (size_t l = 0; l < t.lev.size(); ++l) {
    d.Kp[l] = base + off[k++];
    d.Mp[l] = base + off[k++];
    d.invD[l] = base + off[k++];
    d.Tp[l] = base + off[k++];
    d.TpT[l] = base + off[k++];
    d.S[l] = base + off[k++];
    d.ST[l] = base + off[k++];
    d.Linv[l] = base + off[k++];
  }
  d.Kr = base + off[k++];
  d.Mr = base + off[k++];
  d.Kt = base + off[k++];
  d.Mt = base + off[k++];
  d.W1 = base + off[k++];
  d.Wr = base + off[k++];
}

// concatenated tables (each block padded to 32 entries) and their offsets
inline void flatten_tabs(const Tables &t, std::vector<double> &flat, std::vector<size_t> &off) {
  auto put = [&](const dvec &v) {
    off.push_back(flat.size());
    flat.insert(flat.end(), v.begin(), v.end());
    flat.resize((flat.size() + 31) / 32 * 32 + 32, 0.0);
  };
  for (const PLevel &L : t.lev) {
    put(L.Kp);
    put(L.Mp);
    put(L.invD);
    put(L.Tp);
    put(L.TpT);
    put(L.S);
    put(L.ST);
    put(L.Linv);
  }
  put(t.Kr);
  put(t.Mr);
  put(t.Kt);
  put(t.Mt);
  put(t.W1);
  put(t.Wr);
}

}  // namespace pmg
