// Test infrastructure only (see pch_oracle.cpp's header): the distance oracle.
//
// Sequential Chen-Han with Xin and Wang's improvements (ICH, Section 2 and the
// comparison with ICH in Section 6): windows wait in a priority queue ordered by
// their distance back to the source, every update of geod_dist and angle_split
// takes effect at once, and a child window is dropped by the one-angle-one-split
// rule (Figure 4(a)) or the three-inequality filter (Figure 4(b)).
//
// Windows keep the paper's 6-tuple of Section 3 (Figure 2): (d, A, B, d0, d1, e),
// d0 and d1 being the distances from the start and end vertex of edge e to the
// pseudo-source. This file shares no window arithmetic with the round-based
// reference (pch_oracle.cpp) or the GPU library:
//   * a child's (d0, d1) come straight from its parent's d0, d1 and the apex
//     distance |I v2| - the pseudo-source is never carried into another frame;
//   * the child intervals are the hits of the rays I -> A and I -> B on the
//     opposite edges, from one generic line-segment intersection in the
//     parent's frame;
//   * the filter distances are plain 2-D distances between points of that frame;
//   * the fan of a saddle or boundary vertex (Figure 3(c)) finds its window
//     ends with the law of sines and the standard library's sin;
//   * incoming angles at pseudo-sources come from the triangle (vertex, other
//     edge end, pseudo-source) by Kahan's stable angle formula.
// Only the mesh tables (mesh.cpp) and the readings of the paper (the
// tolerances, which child survives a lost corner, the fan sector) are common.
#include <cmath>
#include <cstring>
#include <queue>
#include <vector>

#include "mesh.h"

namespace {

using orc::OMesh;
using orc::nxt;
using orc::prv;

const double kPi = 3.14159265358979323846;
// "A = v0", "B = v1" and "w occupies v2" (Algorithm 2) hold within this
// fraction of the edge length.
const double kTol = 1e-12;
// A vertex takes a new distance only when it is shorter by more than this
// relative margin, so rounding noise cannot re-trigger it.
const double kImprove = 1.0 - 1e-12;
// A filter drops a window only when the path that beats it is shorter by more
// than this relative margin; near-ties are kept (keeping a window is safe).
const double kMargin = 1.0 + 1e-12;

struct P2 {
  double x, y;
};
inline P2 operator-(P2 a, P2 b) { return {a.x - b.x, a.y - b.y}; }
inline P2 operator+(P2 a, P2 b) { return {a.x + b.x, a.y + b.y}; }
inline P2 operator*(double s, P2 a) { return {s * a.x, s * a.y}; }
inline double cross(P2 a, P2 b) { return a.x * b.y - a.y * b.x; }
inline double dot(P2 a, P2 b) { return a.x * b.x + a.y * b.y; }
inline double dist(P2 a, P2 b) { return std::hypot(a.x - b.x, a.y - b.y); }

// Parameter t of the point P0 + t (P1 - P0) of segment P0 P1 that lies on the
// line through I and Q.
double hit_param(P2 I, P2 Q, P2 P0, P2 P1) {
  const P2 r = Q - I;
  return cross(r, P0 - I) / cross(P1 - P0, r);
}

// Distance from I to the segment [P0, P1].
double seg_dist(P2 I, P2 P0, P2 P1) {
  const P2 u = P1 - P0;
  const double uu = dot(u, u);
  double t = uu > 0.0 ? dot(I - P0, u) / uu : 0.0;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  return dist(I, P0 + t * u);
}

// Angle opposite side c of a triangle with sides a, b, c (Kahan, "Miscalculating
// area and angles of a needle-like triangle"); 0 or pi at the degenerate ends.
double tri_angle(double a, double b, double c) {
  if (a < b) std::swap(a, b);
  const double mu = b >= c ? c - (a - b) : b - (a - c);
  const double num = ((a - b) + c) * mu;
  const double den = (a + (b + c)) * ((a - c) + b);
  if (!(den > 0.0)) return kPi;
  if (!(num > 0.0)) return 0.0;
  return 2.0 * std::atan(std::sqrt(num / den));
}

// The paper's window (Section 3, Figure 2).
struct Win {
  double d;       // distance of the pseudo-source I from the source
  double A, B;    // interval on half-edge e, measured from its start vertex
  double d0, d1;  // |I start(e)|, |I end(e)|
  int32_t e;      // the half-edge; the window looks into face(e)
  int32_t src;    // the vertex the pseudo-source is (the stale test)
};

// Figure 2(b): the pseudo-source in the frame of half-edge e (start at the
// origin, end at (L, 0), face(e) above the axis) is where the circles of radii
// d0 and d1 around the two ends meet, on the side away from face(e).
P2 pseudo_source(double L, double d0, double d1) {
  const double x = 0.5 * (L + (d0 - d1) * (d0 + d1) / L);
  const double h2 = (d0 - x) * (d0 + x);
  return {x, h2 > 0.0 ? -std::sqrt(h2) : 0.0};
}

struct Queued {
  double key;
  int64_t seq;
  Win w;
};
struct Later {
  bool operator()(const Queued& a, const Queued& b) const {
    if (a.key != b.key) return a.key > b.key;
    return a.seq > b.seq;
  }
};

// A distance reaching vertex v, with the angular position (around v, in the
// mesh's CCW corner order) of the direction back along the path.
struct Arrival {
  int32_t v;
  double d, back;
};

struct Ich {
  const OMesh& M;
  double eps;
  bool ch_on, ich_on, full_fan;
  std::vector<double> g;         // geod_dist
  std::vector<double> cD, cX;    // angle_split per corner (oriented edge): apex distance, crossing
  std::priority_queue<Queued, std::vector<Queued>, Later> pq;
  std::vector<Arrival> todo;
  int64_t seq = 0;
  int64_t created = 0, processed = 0, stale = 0, tiny = 0, filtered = 0, updates = 0, corner_updates = 0,
          fans = 0, fan_windows = 0, peak = 0, notwin = 0, deferred = 0;

  Ich(const OMesh& m, double eps_tiny, int32_t filters)
      : M(m), eps(eps_tiny), ch_on(filters & 1), ich_on(filters & 2), full_fan(filters & 4),
        g(m.nv, INFINITY), cD(3 * m.nf, INFINITY), cX(3 * m.nf, 0.0) {}

  void push(const Win& w, double key) {
    pq.push({key, seq++, w});
    created++;
    if ((int64_t)pq.size() > peak) peak = (int64_t)pq.size();
  }

  // Figure 4(b): a window on edge (p, q), made by crossing face edge (q, r),
  // is useless when a path through p, q or r reaches its interval sooner.
  // Bq / Ap are its ends nearest q / p. (Each test at one end covers the whole
  // interval: along the edge the difference of the two path lengths is
  // monotone.) Fan windows have no r.
  bool useless(double d, P2 I, P2 Bq, P2 Ap, P2 p, double gp, P2 q, double gq, const P2* r, double gr) const {
    const double dB = d + dist(I, Bq);
    if (dB > (gp + dist(p, Bq)) * kMargin) return true;
    if (d + dist(I, Ap) > (gq + dist(q, Ap)) * kMargin) return true;
    if (r && dB > (gr + dist(*r, Bq)) * kMargin) return true;
    return false;
  }

  // Fan of windows from pseudo-source vertex v reached at distance d
  // (Figure 3(c)): the directions at least pi away from the incoming one on
  // both sides; every direction at a source (full).
  void fan(int32_t v, double d, double back, bool full) {
    fans++;
    const double Th = M.theta[v];
    for (int32_t q = M.coff[v]; q < M.coff[v + 1]; ++q) {
      const int32_t j = M.corner[q];       // v -> a; the corner spans [phi_j, phi_j + al]
      const int32_t jn = nxt(j), jp = prv(j);  // a -> b, b -> v
      const double al = M.alpha[j];
      double lo, hi;  // part of the corner inside the sector, relative to v -> a
      if (full) {
        lo = 0.0;
        hi = al;
      } else if (!M.bnd[v]) {
        // CCW angle from the incoming direction, folded into [0, Theta)
        double rel = std::fmod(M.phi[j] - back, Th);
        if (rel < 0.0) rel += Th;
        lo = std::max(0.0, kPi - rel);
        hi = std::min(al, (Th - kPi) - rel);
      } else {
        // no wrap around a boundary vertex: |psi - back| >= pi inside [0, Theta]
        const double below = (back - kPi) - M.phi[j];  // psi <= back - pi
        const double above = (back + kPi) - M.phi[j];  // psi >= back + pi
        if (below >= 0.0) {
          lo = 0.0;
          hi = std::min(al, below);
        } else {
          lo = std::max(0.0, above);
          hi = al;
        }
      }
      if (!(lo <= hi)) continue;
      const int32_t a = M.F[jn], b = M.F[jp];
      const double la = M.L[j], lb = M.L[jp], ln = M.L[jn];
      // edge paths along the sector's boundary directions
      if (lo <= 0.0) {
        todo.push_back({a, d + la, M.phi[jn] + M.alpha[jn]});
        deferred++;
      }
      if (hi >= al && M.twin[jp] < 0) {
        todo.push_back({b, d + lb, M.phi[jp]});
        deferred++;
      }
      const int32_t t = M.twin[jn];
      if (t < 0) {
        notwin++;
        continue;
      }
      // law of sines in triangle (v, a, hit): |a hit| = la sin(t) / sin(t + angle at a)
      const double at_a = M.alpha[jn];
      auto from_b = [&](double ang) { return ln - la * std::sin(ang) / std::sin(ang + at_a); };
      double c0 = hi >= al ? 0.0 : from_b(hi);
      double c1 = lo <= 0.0 ? ln : from_b(lo);
      c0 = std::max(c0, 0.0);
      c1 = std::min(c1, ln);
      if (!(c1 - c0 > eps * ln)) {
        tiny++;
        continue;
      }
      // the corner's frame: v at the origin, a on the x axis, b above it
      const P2 pv{0.0, 0.0}, pa{la, 0.0}, pb{lb * std::cos(al), lb * std::sin(al)};
      const P2 H0 = pb + (c0 / ln) * (pa - pb), H1 = pb + (c1 / ln) * (pa - pb);
      // the window on t runs from b to a: H1 is its end nearest a, H0 nearest b
      if (ich_on && useless(d, pv, H1, H0, pb, g[b], pa, g[a], nullptr, 0.0)) {
        filtered++;
        continue;
      }
      push(Win{d, c0, c1, lb, la, t, v}, d + seg_dist(pv, H0, H1));
      fan_windows++;
    }
  }

  // Applies waiting arrivals (and the fans they start) at once.
  void settle() {
    while (!todo.empty()) {
      const Arrival x = todo.back();
      todo.pop_back();
      if (!(x.d < g[x.v] * kImprove)) continue;
      g[x.v] = x.d;
      updates++;
      if (M.pseudo[x.v]) fan(x.v, x.d, x.back, full_fan);
    }
  }

  // One window across face(e) (Algorithm 2 with immediate updates).
  void propagate(const Win& w) {
    const int32_t e = w.e, en = nxt(e), ep = prv(e);
    const double L = M.L[e], tol = kTol * L;
    const int32_t i0 = M.F[e], i1 = M.F[en], i2 = M.F[ep];
    const P2 v0{0.0, 0.0}, v1{L, 0.0}, v2{M.ax[e], M.ay[e]};
    const P2 I = pseudo_source(L, w.d0, w.d1);
    const P2 QA{w.A, 0.0}, QB{w.B, 0.0};
    // where the ray from I through the apex crosses the edge
    const double X = L * hit_param(I, v2, v0, v1);
    const bool occ = X >= w.A - tol && X <= w.B + tol;
    const double D2 = dist(I, v2);
    const double l02 = M.L[ep], l12 = M.L[en];
    if (w.A <= tol) {
      const double back = M.pseudo[i0] ? M.phi[e] - tri_angle(w.d0, L, w.d1) : 0.0;
      todo.push_back({i0, w.d + w.d0, back});
    }
    if (w.B >= L - tol) {
      const double back = M.pseudo[i1] ? (M.phi[en] + M.alpha[en]) + tri_angle(w.d1, L, w.d0) : 0.0;
      todo.push_back({i1, w.d + w.d1, back});
    }
    bool left = false, right = false;
    if (occ) {
      const double back = M.pseudo[i2] ? M.phi[ep] + tri_angle(l02, D2, w.d0) : 0.0;
      todo.push_back({i2, w.d + D2, back});
      const double Dapex = w.d + D2;
      if (!ch_on) {
        left = right = true;
      } else if (Dapex < cD[e]) {
        // Figure 4(a): this window now owns the corner and splits
        corner_updates++;
        cD[e] = Dapex;
        cX[e] = X;
        left = right = true;
      } else if (Dapex <= cD[e] * kMargin) {
        left = right = true;  // a near-tie keeps both children
      } else if (X < cX[e] - tol) {
        left = true;  // the side away from the owner's crossing survives
      } else if (X > cX[e] + tol) {
        right = true;
      } else {
        left = right = true;
      }
    } else if (X > w.B) {
      left = true;
    } else {
      right = true;
    }
    settle();
    // Children: the left one on edge v0 -> v2 (the twin of prev(e)), the right
    // one on edge v2 -> v1 (the twin of next(e)), intervals measured from
    // their start vertex.
    for (int side = 0; side < 2; ++side) {
      if (side == 0 ? !left : !right) continue;
      const int32_t t = M.twin[side == 0 ? ep : en];
      if (t < 0) {
        notwin++;
        continue;
      }
      const P2 s0 = side == 0 ? v0 : v2, s1 = side == 0 ? v2 : v1;
      const double lc = side == 0 ? l02 : l12;
      double t0, t1;
      if (side == 0) {
        t0 = w.A == 0.0 ? 0.0 : hit_param(I, QA, s0, s1);
        t1 = occ ? 1.0 : hit_param(I, QB, s0, s1);
      } else {
        t0 = occ ? 0.0 : hit_param(I, QA, s0, s1);
        t1 = w.B == L ? 1.0 : hit_param(I, QB, s0, s1);
      }
      const double c0 = std::max(t0 * lc, 0.0), c1 = std::min(t1 * lc, lc);
      if (!(c1 - c0 > eps * lc)) {
        tiny++;
        continue;
      }
      const P2 H0 = s0 + (c0 / lc) * (s1 - s0), H1 = s0 + (c1 / lc) * (s1 - s0);
      if (ich_on) {
        // q is the end shared with the parent edge, p the apex, r the other end
        const bool bad = side == 0 ? useless(w.d, I, H0, H1, v2, g[i2], v0, g[i0], &v1, g[i1])
                                   : useless(w.d, I, H1, H0, v2, g[i2], v1, g[i1], &v0, g[i0]);
        if (bad) {
          filtered++;
          continue;
        }
      }
      const Win c = side == 0 ? Win{w.d, c0, c1, w.d0, D2, t, w.src} : Win{w.d, c0, c1, D2, w.d1, t, w.src};
      push(c, w.d + seg_dist(I, H0, H1));
    }
  }

  // max_processed > 0 stops after that many propagated windows (a bounded
  // sample of the run, for timing only: the distances are then incomplete)
  void run(const std::vector<int32_t>& src, int64_t max_processed = 0) {
    for (int32_t s : src) g[s] = 0.0;
    for (int32_t s : src) fan(s, 0.0, 0.0, true);
    settle();
    while (!pq.empty()) {
      if (max_processed > 0 && processed >= max_processed) break;
      const Win w = pq.top().w;
      pq.pop();
      if (w.d > g[w.src]) {
        stale++;
        continue;
      }
      processed++;
      propagate(w);
    }
  }
};

}  // namespace

extern "C" {

// Exact distance field by ICH. filters: bit 0 the one-angle-one-split rule,
// bit 1 the window filter, bit 2 full fans at every pseudo-source. stats
// (int64 [16], nullable): created, processed, stale, tiny, filtered, vertex
// updates, corner updates, fans, fan windows, 0, peak queue, boundary drops,
// edge-path arrivals from fans, 0, 0, 0.
int orc_ich_bounded(const int32_t* faces, int64_t nf, int64_t nv, const double* he_len, const int32_t* src,
                    int32_t m, double eps_tiny, int32_t filters, int64_t max_processed, double* dist_out,
                    int64_t* stats) {
  OMesh M;
  int rc = orc::build_mesh(faces, nf, nv, he_len, M);
  if (rc) return rc;
  std::vector<int32_t> s;
  rc = orc::sorted_sources(src, m, nv, s);
  if (rc) return rc;
  Ich run(M, eps_tiny, filters);
  run.run(s, max_processed);
  for (int64_t v = 0; v < nv; ++v) dist_out[v] = run.g[v];
  if (stats) {
    int64_t st[16] = {run.created, run.processed, run.stale, run.tiny, run.filtered, run.updates,
                      run.corner_updates, run.fans, run.fan_windows, 0, run.peak, run.notwin, run.deferred,
                      0, 0, 0};
    std::memcpy(stats, st, sizeof(st));
  }
  return orc::OK;
}

int orc_ich(const int32_t* faces, int64_t nf, int64_t nv, const double* he_len, const int32_t* src, int32_t m,
            double eps_tiny, int32_t filters, double* dist_out, int64_t* stats) {
  return orc_ich_bounded(faces, nf, nv, he_len, src, m, eps_tiny, filters, 0, dist_out, stats);
}

}  // extern "C"
