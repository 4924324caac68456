// tait.cpp -- knot diagram (PD code) -> signed Tait graph (Sec. II of
// arXiv:1807.02119).
//
// Regions of the diagram are found by walking corners: the wedge at crossing
// i between slots k and k+1 (counter-clockwise) is corner 4i+k.  Leaving
// crossing i along slot k, corner 4i+k lies on the left; at the far end of
// that arc (crossing j, slot p) the same region continues in corner
// 4j+((p+3)&3).  Regions on the two sides of an arc get opposite colours; the
// unbounded region is white (Sec. II).  Black regions are the Tait vertices,
// every crossing joins its two black corners, and the Tait sign is +1 iff the
// region left of the outgoing over-strand is black.
#include <cstring>
#include <new>

#include "internal.h"

namespace {

// Slot of the outgoing over-arc: b for a positive crossing, d for a negative.
inline int out_over_slot(int sign) { return sign > 0 ? 1 : 3; }

// Labels a, b in [0, m): is b the label after a (b = a + 1 mod m)?
inline bool follows(int32_t a, int32_t b, int32_t m) {
  const int32_t d = b - a - 1;
  return d == 0 || d == -m;
}

}  // namespace

extern "C" kn_status kn_build_tait(int32_t n, const int32_t* pd, const int8_t* signs,
                                   int32_t outer_arc, int32_t outer_side, kn_tait** out) {
  if (!out) return KN_E_INVALID;
  *out = nullptr;
  if (n < 0 || (n > 0 && !pd) || n > (1 << 26)) return KN_E_INVALID;
  if (outer_side != 0 && outer_side != 1) return KN_E_INVALID;
  kn_tait* g = new (std::nothrow) kn_tait();
  if (!g) return KN_E_NOMEM;
  if (n == 0) {
    // a single circle: its inside is the one black region
    g->n_vertices = 1;
    *out = g;
    return KN_OK;
  }
  if (n == 1 && !signs) {
    delete g;
    return KN_E_INVALID;
  }
  const int32_t m = 2 * n;
  const int32_t nc = 4 * n;
  try {
    // every arc label used exactly twice: partner[s] is the other slot with
    // the label of slot s.  Without branches: x[lab] is the XOR of the slots
    // carrying lab, so with exactly two of them x[lab] ^ s is the other one.
    std::vector<int32_t> partner(nc), x(m, 0), uses(m, 0);
    uint32_t bad = 0;
    for (int32_t s = 0; s < nc; ++s) {
      const uint32_t lab = (uint32_t)pd[s];
      bad |= (uint32_t)(lab >= (uint32_t)m);
      const uint32_t l = lab < (uint32_t)m ? lab : 0;
      x[l] ^= s;
      uses[l]++;
    }
    for (int32_t lab = 0; lab < m; ++lab) bad |= (uint32_t)(uses[lab] != 2);
    if (bad) { delete g; return KN_E_INVALID; }
    for (int32_t s = 0; s < nc; ++s) partner[s] = x[pd[s]] ^ s;

    // crossing signs and orientation consistency: each label must be the
    // outgoing arc of one slot and the incoming arc of another
    g->twist.resize(n);
    std::vector<uint8_t> n_in(m, 0), n_out(m, 0);
    for (int32_t i = 0; i < n; ++i) {
      const int32_t* x = pd + 4 * i;
      int sg;
      if (signs) {
        sg = signs[i] > 0 ? 1 : (signs[i] < 0 ? -1 : 0);
        if (!sg) { delete g; return KN_E_INVALID; }
      } else {
        bool pos = follows(x[3], x[1], m);
        bool neg = follows(x[1], x[3], m);
        if (pos == neg) { delete g; return KN_E_INVALID; }
        sg = pos ? 1 : -1;
      }
      if (!follows(x[0], x[2], m)) { delete g; return KN_E_INVALID; }
      int oo = out_over_slot(sg), oi = oo ^ 2;
      if (!follows(x[oi], x[oo], m) && n > 1) { delete g; return KN_E_INVALID; }
      g->twist[i] = (int8_t)sg;
      n_in[x[0]]++;
      n_out[x[2]]++;
      n_in[x[oi]]++;
      n_out[x[oo]]++;
    }
    for (int32_t lab = 0; lab < m; ++lab)
      if (n_in[lab] != 1 || n_out[lab] != 1) { delete g; return KN_E_INVALID; }

    // region tracing over corners: corner c continues in corner next(c)
    auto next = [&](int32_t c) {
      const int32_t far = partner[c];
      return (far & ~3) | ((far + 3) & 3);
    };
    std::vector<int32_t> region(nc, -1);
    int32_t nreg = 0;
    for (int32_t c0 = 0; c0 < nc; ++c0) {
      if (region[c0] >= 0) continue;
      int32_t c = c0;
      while (region[c] < 0) {
        region[c] = nreg;
        c = next(c);
      }
      if (c != c0) { delete g; return KN_E_INVALID; }
      ++nreg;
    }
    if (nreg != n + 2) { delete g; return KN_E_INVALID; }  // not a plane diagram

    // two-colouring.  Around a crossing the four corners alternate colours,
    // so crossing i has a parity par[i]: corner slot k is black iff
    // (k & 1) == par[i].  Corners c and next(c) lie in one region, which
    // fixes par of next(c)'s crossing from c's; a breadth-first search over
    // crossings starts from the outer corner, which is white.
    int32_t arc = outer_arc < 0 ? 0 : outer_arc;
    if (arc >= m) { delete g; return KN_E_INVALID; }
    // the slot where `arc` leaves its crossing
    int32_t leave = -1;
    {
      // the two slots carrying `arc`
      int32_t s0 = -1;
      for (int32_t s = 0; s < nc && s0 < 0; ++s)
        if (pd[s] == arc) s0 = s;
      for (int32_t s : {s0, partner[s0]}) {
        int32_t i = s >> 2, k = s & 3;
        if (k == 2 || k == out_over_slot(g->twist[i])) leave = s;
      }
    }
    if (leave < 0) { delete g; return KN_E_INVALID; }
    int32_t outer_corner = outer_side == 0 ? leave : ((leave & ~3) | ((leave + 3) & 3));
    std::vector<int8_t> par(n, -1);
    std::vector<int32_t> queue;
    queue.reserve(n);
    par[outer_corner >> 2] = (int8_t)(1 - (outer_corner & 1));
    queue.push_back(outer_corner >> 2);
    for (size_t h = 0; h < queue.size(); ++h) {
      const int32_t i = queue[h];
      for (int32_t k = 0; k < 4; ++k) {
        const int32_t c = 4 * i + k, d = next(c), j = d >> 2;
        const int8_t pj = (int8_t)(par[i] ^ (c & 1) ^ (d & 1));
        if (par[j] < 0) {
          par[j] = pj;
          queue.push_back(j);
        } else if (par[j] != pj) {
          delete g;
          return KN_E_INVALID;
        }
      }
    }
    if ((int32_t)queue.size() != n) { delete g; return KN_E_INVALID; }  // split diagram
    std::vector<int8_t> colour(nreg, 0);  // 0 white, 1 black
    for (int32_t c = 0; c < nc; ++c) colour[region[c]] = (int8_t)((c & 1) == par[c >> 2]);
    std::vector<int32_t> vid(nreg, -1);
    int32_t nv = 0;
    for (int32_t r = 0; r < nreg; ++r)
      if (colour[r] == 1) vid[r] = nv++;
    g->n_vertices = nv;
    g->uv.resize(2 * n);
    g->eps.resize(n);
    int32_t w = 0, tau = 0;
    for (int32_t i = 0; i < n; ++i) {
      int32_t oo = out_over_slot(g->twist[i]);
      bool left_black = colour[region[4 * i + oo]] == 1;
      // the black corners are the odd ones (1, 3) or the even ones (0, 2)
      int32_t k0 = left_black ? 1 : 0;
      g->uv[2 * i] = vid[region[4 * i + k0]];
      g->uv[2 * i + 1] = vid[region[4 * i + k0 + 2]];
      g->eps[i] = (int8_t)(left_black ? 1 : -1);
      w += g->twist[i];
      tau += g->eps[i];
    }
    g->writhe = w;
    g->tau = tau;
  } catch (const std::bad_alloc&) {
    delete g;
    return KN_E_NOMEM;
  }
  *out = g;
  return KN_OK;
}

extern "C" kn_status kn_tait_info(const kn_tait* g, int32_t* n_vertices, int32_t* n_edges,
                                  int32_t* writhe, int32_t* tait_number) {
  if (!g) return KN_E_INVALID;
  if (n_vertices) *n_vertices = g->n_vertices;
  if (n_edges) *n_edges = (int32_t)g->eps.size();
  if (writhe) *writhe = g->writhe;
  if (tait_number) *tait_number = g->tau;
  return KN_OK;
}

extern "C" kn_status kn_tait_edges(const kn_tait* g, int32_t* uv, int8_t* eps) {
  if (!g) return KN_E_INVALID;
  if (uv && !g->uv.empty()) std::memcpy(uv, g->uv.data(), g->uv.size() * sizeof(int32_t));
  if (eps && !g->eps.empty()) std::memcpy(eps, g->eps.data(), g->eps.size());
  return KN_OK;
}

extern "C" void kn_tait_free(kn_tait* g) { delete g; }
