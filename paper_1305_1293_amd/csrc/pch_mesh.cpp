// Host-side mesh preprocessing for the PCH library (Section 4.1): half-edge
// twins, the per-half-edge unfolding frame, corner angles, the CCW order of
// corners around every vertex and the vertex classes of Section 3
// (boundary, saddle). Runs once per mesh; the result is uploaded to device
// memory by the driver.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "pch.h"
#include "pch_internal.h"

namespace pch {

namespace {

inline int32_t he_next(int32_t j) { return j - j % 3 + (j % 3 + 1) % 3; }
inline int32_t he_prev(int32_t j) { return j - j % 3 + (j % 3 + 2) % 3; }

// 16 * area^2 of a triangle with side lengths p, q, r, by Kahan's
// cancellation-free arrangement of Heron's formula (sides sorted a >= b >= c).
double area16(double p, double q, double r) {
  double s[3] = {p, q, r};
  std::sort(s, s + 3);
  const double a = s[2], b = s[1], c = s[0];
  return (a + (b + c)) * (c - (a - b)) * (c + (a - b)) * (a + (b - c));
}

// Total angle above 2 pi by more than this makes an interior vertex a saddle.
constexpr double kSaddleExcess = 1e-10;
constexpr double kPiHost = 3.14159265358979323846;

}  // namespace

int lengths_from_xyz(const double* xyz, int64_t nv, const int32_t* faces, int64_t nf, std::vector<double>& len,
                     std::string& msg) {
  len.resize(3 * nf);
  for (int64_t j = 0; j < 3 * nf; ++j) {
    const int32_t a = faces[j];
    const int32_t b = faces[he_next((int32_t)j)];
    if (a < 0 || b < 0 || a >= nv || b >= nv) {
      msg = "face index out of range";
      return PCH_EINVAL;
    }
    const double* pa = xyz + 3 * (int64_t)a;
    const double* pb = xyz + 3 * (int64_t)b;
    const double dx = pb[0] - pa[0], dy = pb[1] - pa[1], dz = pb[2] - pa[2];
    len[j] = std::sqrt((dx * dx + dy * dy) + dz * dz);
  }
  return PCH_OK;
}

int build_host_mesh(const int32_t* faces, int64_t nf, int64_t nv, const double* he_len, HostMesh& M,
                    std::string& msg) {
  if (nf < 1 || nv < 1) {
    msg = "mesh needs at least one face and one vertex";
    return PCH_EINVAL;
  }
  if (nf > (int64_t)(INT32_MAX / 3) || nv > (int64_t)INT32_MAX) {
    msg = "mesh too large for 32-bit half-edge indices";
    return PCH_EINVAL;
  }
  const int64_t nh = 3 * nf;
  M.nv = nv;
  M.nf = nf;
  M.nh = nh;
  M.hv.assign(faces, faces + nh);
  for (int64_t f = 0; f < nf; ++f) {
    const int32_t* t = faces + 3 * f;
    for (int i = 0; i < 3; ++i)
      if (t[i] < 0 || t[i] >= nv) {
        msg = "face index out of range";
        return PCH_EINVAL;
      }
    if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) {
      msg = "degenerate face (repeated vertex)";
      return PCH_EMESH;
    }
  }
  for (int64_t j = 0; j < nh; ++j)
    if (!(he_len[j] > 0.0 && he_len[j] < INFINITY)) {
      msg = "half-edge length must be positive and finite";
      return PCH_EINVAL;
    }

  // Twins: sort half-edges by their undirected vertex pair.
  struct Key {
    uint64_t k;
    int32_t j;
  };
  std::vector<Key> keys(nh);
  for (int64_t j = 0; j < nh; ++j) {
    const uint32_t a = (uint32_t)M.hv[j], b = (uint32_t)M.hv[he_next((int32_t)j)];
    keys[j] = {((uint64_t)std::min(a, b) << 32) | (uint64_t)std::max(a, b), (int32_t)j};
  }
  std::sort(keys.begin(), keys.end(), [](const Key& x, const Key& y) { return x.k < y.k || (x.k == y.k && x.j < y.j); });
  M.twin.assign(nh, -1);
  for (int64_t i = 0; i < nh;) {
    int64_t e = i;
    while (e < nh && keys[e].k == keys[i].k) ++e;
    if (e - i > 2) {
      msg = "non-manifold edge shared by more than two faces";
      return PCH_EMESH;
    }
    if (e - i == 2) {
      const int32_t a = keys[i].j, b = keys[i + 1].j;
      if (M.hv[a] == M.hv[b]) {
        msg = "inconsistent face orientation across an edge";
        return PCH_EMESH;
      }
      if (std::fabs(he_len[a] - he_len[b]) > 1e-9 * he_len[a]) {
        msg = "the two half-edges of an edge have different lengths";
        return PCH_EINVAL;
      }
      M.twin[a] = b;
      M.twin[b] = a;
    }
    i = e;
  }

  // Unfolding frame per half-edge.
  M.he.resize(nh);
  M.alpha.resize(nh);
  for (int64_t j = 0; j < nh; ++j) {
    const int32_t n = he_next((int32_t)j), p = he_prev((int32_t)j);
    const double L = he_len[j], l02 = he_len[p], l12 = he_len[n];
    const double a16 = area16(L, l02, l12);
    if (!(a16 > 0.0)) {
      msg = "zero-area face: edge lengths violate the strict triangle inequality";
      return PCH_EMESH;
    }
    HalfEdge& h = M.he[j];
    h.L = L;
    h.l02 = l02;
    h.l12 = l12;
    h.x2 = ((L * L + l02 * l02) - l12 * l12) / (2.0 * L);
    h.y2 = std::sqrt(a16) / (2.0 * L);
    h.v0 = M.hv[j];
    h.v1 = M.hv[n];
    h.v2 = M.hv[p];
    h.tl = -1;
    h.tr = -1;
    h.pflags = 0;
    M.alpha[j] = std::atan2(h.y2, h.x2);
  }
  for (int64_t j = 0; j < nh; ++j) {
    M.he[j].tl = M.twin[he_prev((int32_t)j)];
    M.he[j].tr = M.twin[he_next((int32_t)j)];
  }

  // Corners around each vertex in CCW order: from an outgoing half-edge h the
  // next one counter-clockwise is twin(prev(h)). Boundary vertices start at
  // their outgoing boundary half-edge, interior ones at their smallest index.
  std::vector<int32_t> deg(nv, 0), first(nv, -1), bstart(nv, -1);
  for (int64_t j = 0; j < nh; ++j) {
    const int32_t v = M.hv[j];
    deg[v]++;
    if (first[v] < 0) first[v] = (int32_t)j;
    if (M.twin[j] < 0) {
      if (bstart[v] >= 0) {
        msg = "non-manifold vertex with two boundary gaps";
        return PCH_EMESH;
      }
      bstart[v] = (int32_t)j;
    }
  }
  M.coff.assign(nv + 1, 0);
  for (int64_t v = 0; v < nv; ++v) M.coff[v + 1] = M.coff[v] + deg[v];
  M.corner.assign(nh, -1);
  M.phi.assign(nh, 0.0);
  M.theta.assign(nv, 0.0);
  M.flags.assign(nv, 0);
  M.n_boundary_he = 0;
  for (int64_t j = 0; j < nh; ++j) M.n_boundary_he += M.twin[j] < 0;
  M.n_pseudo = 0;
  const double two_pi = 2.0 * kPiHost;
  for (int64_t v = 0; v < nv; ++v) {
    if (deg[v] == 0) continue;
    const bool boundary = bstart[v] >= 0;
    const int32_t start = boundary ? bstart[v] : first[v];
    int32_t h = start;
    int32_t count = 0;
    double sum = 0.0;
    for (;;) {
      if (count == deg[v]) {
        msg = "non-manifold vertex";
        return PCH_EMESH;
      }
      M.corner[M.coff[v] + count] = h;
      M.phi[h] = sum;
      sum = sum + M.alpha[h];
      ++count;
      const int32_t nxt_h = M.twin[he_prev(h)];
      if (nxt_h < 0 || nxt_h == start) break;
      h = nxt_h;
    }
    if (count != deg[v]) {
      msg = "non-manifold vertex (faces form several fans)";
      return PCH_EMESH;
    }
    M.theta[v] = sum;
    const bool pseudo = boundary || sum > two_pi + kSaddleExcess;
    M.flags[v] = (uint8_t)((boundary ? VF_BOUNDARY : 0) | (pseudo ? VF_PSEUDO : 0));
    M.n_pseudo += pseudo;
  }
  // pseudo-source bits and angular positions per half-edge (after every phi
  // and vertex class is known)
  M.hang.resize(nh);
  for (int64_t j = 0; j < nh; ++j) {
    const int32_t n = he_next((int32_t)j), p = he_prev((int32_t)j);
    HalfEdge& h = M.he[j];
    h.pflags = ((M.flags[h.v0] & VF_PSEUDO) ? 1 : 0) | ((M.flags[h.v1] & VF_PSEUDO) ? 2 : 0) |
               ((M.flags[h.v2] & VF_PSEUDO) ? 4 : 0);
    // the same divisions the propagation would make per window
    M.hang[j] = HalfEdgeAng{M.phi[j],          M.phi[n] + M.alpha[n],  M.phi[p],
                            h.x2 / h.l02,      h.y2 / h.l02,           (h.L - h.x2) / h.l12,
                            (-h.y2) / h.l12,   0.0};
  }
  // corner records (after every phi is known)
  M.crec.resize(nh);
  for (int64_t q = 0; q < nh; ++q) {
    const int32_t j = M.corner[q];
    if (j < 0) continue;
    const int32_t n = he_next(j), p = he_prev(j);
    Corner& c = M.crec[q];
    c.alpha = M.alpha[j];
    c.phi = M.phi[j];
    c.l_va = M.he[j].L;
    c.l_vb = M.he[j].l02;
    c.L = M.he[n].L;
    c.x2 = M.he[n].x2;
    c.y2 = M.he[n].y2;
    c.th_a = M.phi[n] + M.alpha[n];
    c.th_b = M.phi[p];
    c.a = M.hv[n];
    c.b = M.hv[p];
    c.tw = M.twin[n];
    c.last = M.twin[p] < 0 ? 1 : 0;
  }
  return PCH_OK;
}

}  // namespace pch
