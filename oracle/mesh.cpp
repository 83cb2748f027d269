// Test infrastructure only (see pch_oracle.cpp's header): mesh tables shared by
// the two CPU references, edge lengths from coordinates, and Dijkstra along mesh
// edges (an upper bound of every geodesic distance).
#include "mesh.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <queue>
#include <unordered_map>

namespace orc {

namespace {
thread_local std::string g_err;
const double kTwoPi = 2.0 * 3.14159265358979323846;
}  // namespace

int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

const char* last_error() { return g_err.c_str(); }

int sorted_sources(const int32_t* src, int32_t m, int64_t nv, std::vector<int32_t>& out) {
  if (m <= 0) return fail(EINVAL_, "no source vertex");
  for (int32_t i = 0; i < m; ++i)
    if (src[i] < 0 || src[i] >= nv) return fail(EINVAL_, "source vertex out of range");
  out.assign(src, src + m);
  std::sort(out.begin(), out.end());
  out.erase(std::unique(out.begin(), out.end()), out.end());
  return OK;
}

// Kahan's stable form of Heron's formula: 16 area^2 with sides a >= b >= c.
double kahan16(double p, double q, double r) {
  double a = p, b = q, c = r;
  if (a < b) std::swap(a, b);
  if (b < c) std::swap(b, c);
  if (a < b) std::swap(a, b);
  return (a + (b + c)) * (c - (a - b)) * (c + (a - b)) * (a + (b - c));
}

int build_mesh(const int32_t* faces, int64_t nf, int64_t nv, const double* len, OMesh& M) {
  if (nf <= 0 || nv <= 0) return fail(EINVAL_, "empty mesh");
  if (3 * nf > (int64_t)INT32_MAX) return fail(EINVAL_, "too many faces");
  M.nv = nv;
  M.nf = nf;
  const int64_t nh = 3 * nf;
  M.F.assign(faces, faces + nh);
  M.L.assign(len, len + nh);
  for (int64_t f = 0; f < nf; ++f) {
    int32_t a = faces[3 * f], b = faces[3 * f + 1], c = faces[3 * f + 2];
    if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) return fail(EINVAL_, "face index out of range");
    if (a == b || b == c || a == c) return fail(EMESH, "face with a repeated vertex");
  }
  for (int64_t j = 0; j < nh; ++j)
    if (!(M.L[j] > 0.0) || !std::isfinite(M.L[j])) return fail(EINVAL_, "edge length not positive and finite");
  // twins by (min, max) vertex pair
  M.twin.assign(nh, -1);
  std::unordered_map<uint64_t, int32_t> first;
  first.reserve(nh * 2);
  std::vector<uint8_t> paired(nh, 0);
  for (int64_t j = 0; j < nh; ++j) {
    uint32_t a = (uint32_t)M.F[j], b = (uint32_t)M.F[nxt((int32_t)j)];
    uint64_t key = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
    auto it = first.find(key);
    if (it == first.end()) {
      first.emplace(key, (int32_t)j);
    } else {
      int32_t o = it->second;
      if (o < 0) return fail(EMESH, "non-manifold edge (more than two faces)");
      if (M.F[o] == M.F[j]) return fail(EMESH, "inconsistent face orientation");
      M.twin[j] = o;
      M.twin[o] = (int32_t)j;
      it->second = -1;
    }
  }
  for (int64_t j = 0; j < nh; ++j) {
    int32_t t = M.twin[j];
    if (t >= 0 && std::fabs(M.L[j] - M.L[t]) > 1e-9 * M.L[j]) return fail(EINVAL_, "twin half-edges differ in length");
  }
  // apex coordinates and corner angles
  M.ax.resize(nh);
  M.ay.resize(nh);
  M.alpha.resize(nh);
  for (int64_t j = 0; j < nh; ++j) {
    double Lj = M.L[j], lp = M.L[prv((int32_t)j)], ln = M.L[nxt((int32_t)j)];
    double P = kahan16(Lj, lp, ln);
    if (!(P > 0.0)) return fail(EMESH, "zero-area face (triangle inequality not strict)");
    M.ax[j] = ((Lj * Lj + lp * lp) - ln * ln) / (2.0 * Lj);
    M.ay[j] = std::sqrt(P) / (2.0 * Lj);
    M.alpha[j] = std::atan2(M.ay[j], M.ax[j]);
  }
  // CCW order of outgoing half-edges around every vertex
  std::vector<int32_t> cnt(nv, 0), bstart(nv, -1), mn(nv, INT32_MAX);
  for (int64_t j = 0; j < nh; ++j) {
    int32_t v = M.F[j];
    cnt[v]++;
    if (j < mn[v]) mn[v] = (int32_t)j;
    if (M.twin[j] < 0) {
      if (bstart[v] >= 0) return fail(EMESH, "non-manifold vertex (two boundary fans)");
      bstart[v] = (int32_t)j;
    }
  }
  M.coff.assign(nv + 1, 0);
  for (int64_t v = 0; v < nv; ++v) M.coff[v + 1] = M.coff[v] + cnt[v];
  M.corner.assign(nh, -1);
  M.phi.assign(nh, 0.0);
  M.theta.assign(nv, 0.0);
  M.bnd.assign(nv, 0);
  M.pseudo.assign(nv, 0);
  for (int64_t v = 0; v < nv; ++v) {
    if (cnt[v] == 0) continue;
    int32_t h0 = bstart[v] >= 0 ? bstart[v] : mn[v];
    M.bnd[v] = bstart[v] >= 0;
    int32_t h = h0, k = 0;
    double acc = 0.0;
    while (true) {
      if (k >= cnt[v]) return fail(EMESH, "non-manifold vertex");
      M.corner[M.coff[v] + k] = h;
      M.phi[h] = acc;
      acc = acc + M.alpha[h];
      ++k;
      int32_t t = M.twin[prv(h)];
      if (t < 0 || t == h0) break;
      h = t;
    }
    if (k != cnt[v]) return fail(EMESH, "non-manifold vertex (several fans)");
    M.theta[v] = acc;
    M.pseudo[v] = M.bnd[v] || (acc > kTwoPi + kSaddle);
  }
  return OK;
}

}  // namespace orc

using namespace orc;

extern "C" {

const char* orc_last_error(void) { return last_error(); }

// Half-edge lengths from coordinates: sqrt((dx*dx + dy*dy) + dz*dz), with
// d = xyz[end] - xyz[start].
int orc_lengths(const double* xyz, int64_t nv, const int32_t* faces, int64_t nf, double* he_len) {
  for (int64_t f = 0; f < nf; ++f) {
    for (int i = 0; i < 3; ++i) {
      int32_t a = faces[3 * f + i], b = faces[3 * f + (i + 1) % 3];
      if (a < 0 || b < 0 || a >= nv || b >= nv) return fail(EINVAL_, "face index out of range");
      double dx = xyz[3 * b] - xyz[3 * a];
      double dy = xyz[3 * b + 1] - xyz[3 * a + 1];
      double dz = xyz[3 * b + 2] - xyz[3 * a + 2];
      he_len[3 * f + i] = std::sqrt((dx * dx + dy * dy) + dz * dz);
    }
  }
  return OK;
}

// Mesh tables for tests: twin[3nf], ax/ay/alpha/phi[3nf], theta[nv], flags[nv]
// (bit 0 boundary, bit 1 pseudo-source).
int orc_mesh_info(const int32_t* faces, int64_t nf, int64_t nv, const double* he_len, int32_t* twin, double* ax,
                  double* ay, double* alpha, double* phi, double* theta, uint8_t* flags) {
  OMesh M;
  int rc = build_mesh(faces, nf, nv, he_len, M);
  if (rc) return rc;
  const int64_t nh = 3 * nf;
  for (int64_t j = 0; j < nh; ++j) {
    twin[j] = M.twin[j];
    ax[j] = M.ax[j];
    ay[j] = M.ay[j];
    alpha[j] = M.alpha[j];
    phi[j] = M.phi[j];
  }
  for (int64_t v = 0; v < nv; ++v) {
    theta[v] = M.theta[v];
    flags[v] = (uint8_t)(M.bnd[v] | (M.pseudo[v] << 1));
  }
  return OK;
}

// Dijkstra along mesh edges (length of the best edge path).
int orc_dijkstra(const int32_t* faces, int64_t nf, int64_t nv, const double* he_len, const int32_t* src, int32_t m,
                 double* dist) {
  std::vector<int32_t> s;
  int rc = sorted_sources(src, m, nv, s);
  if (rc) return rc;
  std::vector<std::vector<std::pair<int32_t, double>>> adj(nv);
  for (int64_t j = 0; j < 3 * nf; ++j) {
    int32_t a = faces[j], b = faces[nxt((int32_t)j)];
    adj[a].push_back({b, he_len[j]});
    adj[b].push_back({a, he_len[j]});
  }
  for (int64_t v = 0; v < nv; ++v) dist[v] = INFINITY;
  typedef std::pair<double, int32_t> QE;
  std::priority_queue<QE, std::vector<QE>, std::greater<QE>> q;
  for (int32_t i = 0; i < m; ++i) {
    dist[src[i]] = 0.0;
    q.push({0.0, src[i]});
  }
  while (!q.empty()) {
    QE t = q.top();
    q.pop();
    if (t.first > dist[t.second]) continue;
    for (auto& e : adj[t.second]) {
      double nd = t.first + e.second;
      if (nd < dist[e.first]) {
        dist[e.first] = nd;
        q.push({nd, e.first});
      }
    }
  }
  return OK;
}

}  // extern "C"
