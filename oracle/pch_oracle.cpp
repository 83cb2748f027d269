// Test infrastructure only: plain, slow CPU references for exact geodesic
// distance on triangle meshes (Ying, Xin, He: "Parallel Chen-Han (PCH)
// Algorithm for Discrete Geodesics"). Only the test suite, the smoke check and
// the benchmark's CPU-baseline leg load this library (liboracle.so, built from
// this file, ich.cpp and mesh.cpp). The GPU library shares no code with it.
//
// The library holds:
//   * ich      (ich.cpp) - sequential Chen-Han with Xin and Wang's priority
//                queue and window filter, windows in the paper's (d, A, B, d0,
//                d1, e) form, immediate updates: the distance oracle;
//   * replica  (this file) - the round-based PCH method (Algorithm 1) run
//                sequentially: select all windows whose key is at or below a
//                cutoff, propagate them against the round-start state (delayed
//                update, Remark 3), then apply the distance and angle events by
//                minimum (Algorithm 4). Windows keep their pseudo-source as
//                (px, py) in the edge frame. It logs per-round integer counts,
//                the record the GPU's rounds are compared with;
//   * mesh tables and Dijkstra along edges (mesh.cpp), used by both.
// The two window codes share no function: each has its own propagation, fan,
// filter and key.
//
// Floating point: built with -ffp-contract=off and no fast-math. sqrt and
// division are IEEE correctly rounded. The replica's atan2, sin and cos are
// this file's own series (stated below), evaluated in the same order as the
// GPU library's, so that the two take every floating-point decision alike and
// their per-round records can be compared exactly.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <queue>
#include <string>
#include <unordered_map>
#include <vector>

#include "mesh.h"

using namespace orc;

namespace {

const double kPi = 3.14159265358979323846;
const double kHalfPi = 0.5 * 3.14159265358979323846;
const double kQuarterPi = 0.25 * 3.14159265358979323846;
// Relative tolerance for "A = v0", "B = v1" and "w occupies v2" (Algorithm 2).
const double kTau = 1e-12;
// A distance event is raised only when it lowers geod_dist by more than a
// relative 1e-12 (d < g * kEv), so rounding noise cannot re-trigger a vertex.
const double kEv = 1.0 - 1e-12;
// Filters drop a window only when the dominating path is shorter by more than
// a relative 1e-12: near-ties are left to rounding otherwise, and a window
// grazing a nearly straight convex boundary vertex (the only one carrying rays
// past it) can lose a tie it wins in exact arithmetic.
const double kFm = 1.0 + 1e-12;

// --------------------------------------------------------------------------
// own elementary functions (only + - * / sqrt, fixed order)
// --------------------------------------------------------------------------

// atan on [0, 1]: two half-angle steps, atan(t) = 2 atan(t / (1 + sqrt(1 + t^2))),
// bring the argument to at most tan(pi/16); then the Maclaurin series of atan
// with 13 terms, summed by Horner in u^2.
double orc_atan01(double t) {
  double u = t / (1.0 + std::sqrt(1.0 + t * t));
  u = u / (1.0 + std::sqrt(1.0 + u * u));
  double u2 = u * u;
  double p = 0.0;
  for (int i = 12; i >= 0; --i) {
    double c = 1.0 / (double)(2 * i + 1);
    if (i & 1) c = -c;
    p = p * u2 + c;
  }
  return 4.0 * (u * p);
}

double orc_atan2(double y, double x) {
  double ax = std::fabs(x), ay = std::fabs(y);
  if (ax == 0.0 && ay == 0.0) return 0.0;
  double r;
  if (ay > ax) {
    r = kHalfPi - orc_atan01(ax / ay);
  } else {
    r = orc_atan01(ay / ax);
  }
  if (x < 0.0) r = kPi - r;
  if (y < 0.0) r = -r;
  return r;
}

// sin and cos of t in [0, pi]: fold to [0, pi/4] by symmetry, then nested
// Maclaurin series (11 factors each, multiplying by the factors' reciprocals).
void orc_sincos01(double u, double* s, double* c) {
  double u2 = u * u;
  double ps = 1.0, pc = 1.0;
  for (int n = 11; n >= 1; --n) {
    double rs = 1.0 / ((double)(2 * n) * (double)(2 * n + 1));
    double rc = 1.0 / ((double)(2 * n - 1) * (double)(2 * n));
    ps = 1.0 - (u2 * rs) * ps;
    pc = 1.0 - (u2 * rc) * pc;
  }
  *s = u * ps;
  *c = pc;
}

void orc_sincos(double t, double* s, double* c) {
  double sgn_c = 1.0;
  if (t > kHalfPi) {
    t = kPi - t;
    sgn_c = -1.0;
  }
  double ss, cc;
  if (t > kQuarterPi) {
    orc_sincos01(kHalfPi - t, &cc, &ss);
  } else {
    orc_sincos01(t, &ss, &cc);
  }
  *s = ss;
  *c = sgn_c * cc;
}

// --------------------------------------------------------------------------
// window geometry of the replica (Section 3, Algorithm 2)
// --------------------------------------------------------------------------

struct Ev {
  int32_t v;
  double d, th;  // distance, angular position of the incoming ray's back direction
};
struct AEv {
  int32_t e;
  double D, X;
};
struct Cand {
  int32_t e, src;
  double b0, b1, px, py, sg, key, d0, d1;
};
struct Cnt {
  int64_t tiny = 0, ich = 0, notwin = 0, kept = 0, dist_ev = 0, ang_ev = 0, fans = 0, fan_kept = 0, deferred = 0;
};

double key_of(double b0, double b1, double px, double py, double sg) {
  double dseg;
  if (px < b0) {
    double dx = b0 - px;
    dseg = std::sqrt(dx * dx + py * py);
  } else if (px > b1) {
    double dx = px - b1;
    dseg = std::sqrt(dx * dx + py * py);
  } else {
    dseg = -py;
  }
  return sg + dseg;
}

// Distances of a child's endpoints are tested against the endpoint vertices
// (u0 at c1, u1 at c0) and, for children made by crossing a face, against the
// third vertex r at the endpoint next to the shared vertex (Figure 4(b)).
bool child_filter(double c0, double c1, double cpx, double cpy, double sg, double lc, double gu0, double gu1,
                  bool rtest, bool r_at_c0, double gr, double rdist, double eps_tiny, bool ich_on, Cnt& C) {
  if (!(c1 - c0 > eps_tiny * lc)) {
    C.tiny++;
    return false;
  }
  if (!ich_on) return true;
  double dx1 = c1 - cpx;
  double f1 = sg + std::sqrt(dx1 * dx1 + cpy * cpy);
  if (f1 > (gu0 + c1) * kFm) {
    C.ich++;
    return false;
  }
  double dx0 = c0 - cpx;
  double f0 = sg + std::sqrt(dx0 * dx0 + cpy * cpy);
  if (f0 > (gu1 + (lc - c0)) * kFm) {
    C.ich++;
    return false;
  }
  if (rtest) {
    double lhs = r_at_c0 ? f0 : f1;
    if (lhs > (gr + rdist) * kFm) {
      C.ich++;
      return false;
    }
  }
  return true;
}

// Propagate one window (pseudo-source (px, py) in the frame of half-edge e)
// across face(e) against the state (g, AD, AX). Children are appended to kids,
// events to dev and aev; nothing in the state is written.
// retest (stronger filtering, the paper's first item of future work): before
// it crosses the face, the window takes the two endpoint tests of the ICH
// filter (Figure 4(b)) again with the current g. Along the window's edge
// |I x| - |v0 x| never increases toward v1 and |I x| - |v1 x| never increases
// toward v0, whatever the pseudo-source I, so a window that fails a test at
// the endpoint where that difference is smallest is beaten on its whole
// interval by a path through v0 or v1; it is counted with the ICH drops.
void propagate(const OMesh& M, double b0, double b1, double px, double py, double sg, int32_t e, int32_t src,
               const double* g, const double* AD, const double* AX, bool ch_on, bool ich_on, bool retest,
               double eps_tiny, std::vector<Ev>& dev, std::vector<AEv>& aev, std::vector<Cand>& kids, Cnt& C) {
  const int32_t en = nxt(e), ep = prv(e);
  const double L = M.L[e], x2 = M.ax[e], y2 = M.ay[e];
  const double l02 = M.L[ep], l12 = M.L[en];
  const int32_t v0 = M.F[e], v1 = M.F[en], v2 = M.F[ep];
  const int32_t tl = M.twin[ep], tr = M.twin[en];
  const double g0 = g[v0], g1 = g[v1], g2 = g[v2];
  const double tol = kTau * L;
  if (retest) {
    // at b1 against v0 (distance along the edge b1), at b0 against v1
    double dx1 = b1 - px;
    double f1 = sg + std::sqrt(dx1 * dx1 + py * py);
    double dx0 = b0 - px;
    double f0 = sg + std::sqrt(dx0 * dx0 + py * py);
    if (f1 > (g0 + b1) * kFm || f0 > (g1 + (L - b0)) * kFm) {
      C.ich++;
      return;
    }
  }

  const double den = y2 - py;
  const double t = (-py) / den;
  const double X = px + (x2 - px) * t;
  const bool occ = (X >= b0 - tol) && (X <= b1 + tol);

  if (b0 <= tol) {
    double d = sg + std::sqrt(px * px + py * py);
    if (d < g0 * kEv) {
      double th = M.pseudo[v0] ? M.phi[e] - orc_atan2(-py, px) : 0.0;
      dev.push_back({v0, d, th});
      C.dist_ev++;
    }
  }
  if (b1 >= L - tol) {
    double dx = px - L;
    double d = sg + std::sqrt(dx * dx + py * py);
    if (d < g1 * kEv) {
      double th = M.pseudo[v1] ? (M.phi[en] + M.alpha[en]) + orc_atan2(-py, L - px) : 0.0;
      dev.push_back({v1, d, th});
      C.dist_ev++;
    }
  }
  bool doL = false, doR = false;
  if (occ) {
    double dx = x2 - px, dy = y2 - py;
    double d2 = sg + std::sqrt(dx * dx + dy * dy);
    if (d2 < g2 * kEv) {
      double th = 0.0;
      if (M.pseudo[v2]) {
        double ux = -x2, uy = -y2, wx = px - x2, wy = py - y2;
        double cr = ux * wy - uy * wx;
        double dt = ux * wx + uy * wy;
        th = M.phi[ep] + orc_atan2(cr, dt);
      }
      dev.push_back({v2, d2, th});
      C.dist_ev++;
    }
    if (!ch_on) {
      doL = doR = true;
    } else {
      double Ds = AD[e], Xs = AX[e];
      if (d2 < Ds) {
        aev.push_back({e, d2, X});
        C.ang_ev++;
        doL = doR = true;
      } else if (d2 <= Ds * kFm) {
        doL = doR = true;  // a near-tie keeps both children
      } else if (X < Xs - tol) {
        doL = true;
      } else if (X > Xs + tol) {
        doR = true;
      } else {
        doL = doR = true;
      }
    }
  } else if (X > b1) {
    doL = true;
  } else {
    doR = true;
  }

  if (doL) {
    if (tl < 0) {
      C.notwin++;
    } else {
      double s0, s1;
      if (b0 == 0.0) {
        s0 = 0.0;
      } else {
        double dn0 = x2 * py + y2 * (b0 - px);
        s0 = (py * b0) / dn0;
      }
      if (occ) {
        s1 = 1.0;
      } else {
        double dn1 = x2 * py + y2 * (b1 - px);
        s1 = (py * b1) / dn1;
      }
      double c0 = s0 * l02, c1 = s1 * l02;
      if (c0 < 0.0) c0 = 0.0;
      if (c1 > l02) c1 = l02;
      double ux = x2 / l02, uy = y2 / l02;
      double cpx = ux * px + uy * py;
      double cpy = ux * py - uy * px;
      if (cpy > 0.0) cpy = 0.0;
      double rx = ux * c0 - L, ry = uy * c0;
      double rdist = std::sqrt(rx * rx + ry * ry);
      if (child_filter(c0, c1, cpx, cpy, sg, l02, g0, g2, true, true, g1, rdist, eps_tiny, ich_on, C)) {
        Cand k;
        k.e = tl;
        k.src = src;
        k.b0 = c0;
        k.b1 = c1;
        k.px = cpx;
        k.py = cpy;
        k.sg = sg;
        k.key = key_of(c0, c1, cpx, cpy, sg);
        k.d0 = std::sqrt(px * px + py * py);
        double qx = x2 - px, qy = y2 - py;
        k.d1 = std::sqrt(qx * qx + qy * qy);
        kids.push_back(k);
        C.kept++;
      }
    }
  }
  if (doR) {
    if (tr < 0) {
      C.notwin++;
    } else {
      const double ex = L - x2;
      double r0, r1;
      if (occ) {
        r0 = 0.0;
      } else {
        double nm0 = (x2 * py - py * b0) + y2 * (b0 - px);
        double dn0 = y2 * (b0 - px) - ex * py;
        r0 = nm0 / dn0;
      }
      if (b1 == L) {
        r1 = 1.0;
      } else {
        double nm1 = (x2 * py - py * b1) + y2 * (b1 - px);
        double dn1 = y2 * (b1 - px) - ex * py;
        r1 = nm1 / dn1;
      }
      double c0 = r0 * l12, c1 = r1 * l12;
      if (c0 < 0.0) c0 = 0.0;
      if (c1 > l12) c1 = l12;
      double ux = ex / l12, uy = (-y2) / l12;
      double qx = px - x2, qy = py - y2;
      double cpx = ux * qx + uy * qy;
      double cpy = ux * qy - uy * qx;
      if (cpy > 0.0) cpy = 0.0;
      double rx = x2 + ux * c1, ry = y2 + uy * c1;
      double rdist = std::sqrt(rx * rx + ry * ry);
      if (child_filter(c0, c1, cpx, cpy, sg, l12, g2, g1, true, false, g0, rdist, eps_tiny, ich_on, C)) {
        Cand k;
        k.e = tr;
        k.src = src;
        k.b0 = c0;
        k.b1 = c1;
        k.px = cpx;
        k.py = cpy;
        k.sg = sg;
        k.key = key_of(c0, c1, cpx, cpy, sg);
        double wx = x2 - px, wy = y2 - py;
        k.d0 = std::sqrt(wx * wx + wy * wy);
        double zx = L - px;
        k.d1 = std::sqrt(zx * zx + py * py);
        kids.push_back(k);
        C.kept++;
      }
    }
  }
}

// Windows from a pseudo-source vertex v reached at distance d (Figure 3(c)):
// one window on the far side of every face edge opposite v whose corner meets
// the sector of directions that keep an angle of at least pi to the incoming
// ray on both sides (the MMP theorem, Section 3). full = every direction
// (used for sources). Endpoint vertices in the sector get deferred events.
void fan(const OMesh& M, int32_t v, double d, double th, bool full, const double* g, double eps_tiny, bool ich_on,
         std::vector<Cand>& wins, std::vector<Ev>& deferred, Cnt& C) {
  const double Th = M.theta[v];
  const bool bd = M.bnd[v];
  C.fans++;
  for (int32_t q = M.coff[v]; q < M.coff[v + 1]; ++q) {
    const int32_t j = M.corner[q];
    const double al = M.alpha[j];
    double t0, t1;
    if (full) {
      t0 = 0.0;
      t1 = al;
    } else if (!bd) {
      double rel = M.phi[j] - th;
      if (!std::isfinite(rel)) continue;
      while (rel < 0.0) rel += Th;
      while (rel >= Th) rel -= Th;
      double lo = kPi - rel;
      double hi = (Th - kPi) - rel;
      t0 = lo > 0.0 ? lo : 0.0;
      t1 = hi < al ? hi : al;
      if (!(t0 <= t1)) continue;
    } else {
      double rel = M.phi[j] - th;
      double hiA = -kPi - rel;
      double loB = kPi - rel;
      if (hiA >= 0.0) {
        t0 = 0.0;
        t1 = hiA < al ? hiA : al;
      } else if (loB <= al) {
        t0 = loB > 0.0 ? loB : 0.0;
        t1 = al;
      } else {
        continue;
      }
    }
    const int32_t n = nxt(j), pj = prv(j);
    const int32_t a = M.F[n], b = M.F[pj];
    if (t0 <= 0.0) {
      double da = d + M.L[j];
      if (da < g[a] * kEv) {
        deferred.push_back({a, da, M.phi[n] + M.alpha[n]});
        C.deferred++;
      }
    }
    if (t1 >= al && M.twin[pj] < 0) {
      double db = d + M.L[pj];
      if (db < g[b] * kEv) {
        deferred.push_back({b, db, M.phi[pj]});
        C.deferred++;
      }
    }
    const int32_t tw = M.twin[n];
    if (tw < 0) {
      C.notwin++;
      continue;
    }
    const double Ln = M.L[n], x2n = M.ax[n], y2n = M.ay[n];
    const double ipx = Ln - x2n, ipy = -y2n;
    double c0, c1;
    if (t1 >= al) {
      c0 = 0.0;
    } else {
      double s, c;
      orc_sincos(t1, &s, &c);
      double dx = c * x2n - s * y2n, dy = s * x2n + c * y2n;
      c0 = ipx - ipy * (dx / dy);
    }
    if (t0 <= 0.0) {
      c1 = Ln;
    } else {
      double s, c;
      orc_sincos(t0, &s, &c);
      double dx = c * x2n - s * y2n, dy = s * x2n + c * y2n;
      c1 = ipx - ipy * (dx / dy);
    }
    if (c0 < 0.0) c0 = 0.0;
    if (c1 > Ln) c1 = Ln;
    // endpoints: tw runs from b (u0) to a (u1)
    if (!child_filter(c0, c1, ipx, ipy, d, Ln, g[b], g[a], false, false, 0.0, 0.0, eps_tiny, ich_on, C)) continue;
    Cand k;
    k.e = tw;
    k.src = v;
    k.b0 = c0;
    k.b1 = c1;
    k.px = ipx;
    k.py = ipy;
    k.sg = d;
    k.key = key_of(c0, c1, ipx, ipy, d);
    k.d0 = M.L[pj];
    k.d1 = M.L[j];
    wins.push_back(k);
    C.fan_kept++;
  }
}

// --------------------------------------------------------------------------
// replica: round-based PCH with delayed updates
// --------------------------------------------------------------------------

inline uint64_t bits_of(double x) {
  uint64_t u;
  std::memcpy(&u, &x, 8);
  return u;
}

// Round cutoff: keys (non-negative doubles) compared as uint64 bit patterns.
// With mn, mx the smallest and largest pattern and p the highest bit where they
// differ, patterns are truncated by s = max(p + 1 - 36, 0) bits; the cutoff is
// the k-th smallest truncated value T (1-based) and a window is selected when
// its truncated key is <= T. If N <= k every window is selected.
struct Cut {
  bool all;
  int shift;
  uint64_t T;
};

Cut pick_cutoff(const std::vector<double>& keys, int64_t k) {
  Cut c{true, 0, 0};
  const int64_t N = (int64_t)keys.size();
  if (N <= k) return c;
  uint64_t mn = UINT64_MAX, mx = 0;
  for (double x : keys) {
    uint64_t u = bits_of(x);
    mn = std::min(mn, u);
    mx = std::max(mx, u);
  }
  c.all = false;
  uint64_t dif = mn ^ mx;
  if (dif == 0) {
    c.shift = 0;
    c.T = mx;
    return c;
  }
  int p = 63 - __builtin_clzll(dif);
  int s = p + 1 - 36;
  if (s < 0) s = 0;
  std::vector<uint64_t> t(N);
  for (int64_t i = 0; i < N; ++i) t[i] = bits_of(keys[i]) >> s;
  std::nth_element(t.begin(), t.begin() + (k - 1), t.end());
  c.shift = s;
  c.T = t[k - 1];
  return c;
}

struct RWin {
  double b0, b1, px, py, sg, key;
  int32_t e, src;
};

// round log record (int64 each)
enum {
  RL_N = 0, RL_CUTBITS, RL_SHIFT, RL_SEL, RL_STALE, RL_KIDS, RL_TINY, RL_ICH, RL_DEV, RL_AEV, RL_FANS, RL_FANWIN,
  RL_DEFER, RL_NEND, RL_WIDTH
};

// Selection rules of the replica: 0 = k-th smallest key (pick_cutoff);
// 1 = adaptive step: with m the smallest key in the pool, select keys <= m + delta;
// after a round that did not take the whole pool, delta is multiplied by
// k / selected clamped to [1/2, 2]. A cutoff table overrides either rule for
// its rounds.
int run_replica(const OMesh& M, const int32_t* src, int32_t m, int64_t k, int32_t hops, double eps_tiny,
                int32_t filters, int32_t mode, double delta0, const double* cut_table, int64_t n_cut, double* dist,
                int64_t* stats, int64_t* rlog, int64_t max_log, int64_t* n_rounds, int64_t* vupd) {
  const bool ch_on = filters & 1, ich_on = filters & 2, full_fan = filters & 4;
  const bool retest = (filters & 8) != 0;
  const int64_t nh = 3 * M.nf;
  std::vector<double> g(M.nv, INFINITY), AD(nh, INFINITY), AX(nh, 0.0);
  std::vector<RWin> pool, nextp;
  std::vector<Ev> pending, dev, dfr;
  std::vector<AEv> aev;
  std::vector<Cand> kids, fw, hop_in;
  std::vector<double> fan_th(M.nv, INFINITY);
  std::vector<int32_t> touched;
  Cnt Ctot;
  int64_t created = 0, processed = 0, stale_tot = 0, peak = 0, rounds = 0, updates = 0, ang_updates = 0;
  double delta = delta0;

  auto add = [&](std::vector<RWin>& P, const std::vector<Cand>& ks) {
    for (const Cand& c : ks) P.push_back({c.b0, c.b1, c.px, c.py, c.sg, c.key, c.e, c.src});
    created += (int64_t)ks.size();
  };

  for (int32_t i = 0; i < m; ++i) g[src[i]] = 0.0;
  {
    Cnt C;
    for (int32_t i = 0; i < m; ++i) fan(M, src[i], 0.0, 0.0, true, g.data(), eps_tiny, ich_on, fw, pending, C);
    add(pool, fw);
    fw.clear();
  }
  while (!pool.empty() || !pending.empty()) {
    Cnt C;
    const int64_t N = (int64_t)pool.size();
    peak = std::max(peak, N);
    std::vector<double> keys(N);
    for (int64_t i = 0; i < N; ++i) keys[i] = pool[i].key;
    bool ext = cut_table != nullptr && rounds < n_cut;
    const bool dmode = !ext && mode == 1 && N > k;
    Cut cut{true, 0, 0};
    double cval = INFINITY;
    if (ext) {
      cval = cut_table[rounds];
    } else if (dmode) {
      double mn = INFINITY;
      for (double x : keys) mn = x < mn ? x : mn;
      cval = mn + delta;
    } else if (mode == 1) {
      cut.all = true;
    } else {
      cut = pick_cutoff(keys, k);
    }
    nextp.clear();
    dev.clear();
    aev.clear();
    kids.clear();
    int64_t nsel = 0, nstale = 0;
    // this round's selection test on a key
    auto selected = [&](double key) {
      if (ext || dmode) return key <= cval;
      return cut.all || ((bits_of(key) >> cut.shift) <= cut.T);
    };
    // snapshot semantics: every selected window reads the same g, AD, AX
    for (int64_t i = 0; i < N; ++i) {
      const RWin& w = pool[i];
      if (w.sg > g[w.src]) {
        nstale++;
        continue;
      }
      if (!selected(w.key)) {
        nextp.push_back(w);
        continue;
      }
      nsel++;
      propagate(M, w.b0, w.b1, w.px, w.py, w.sg, w.e, w.src, g.data(), AD.data(), AX.data(), ch_on, ich_on, retest,
                eps_tiny, dev, aev, kids, C);
    }
    // Further hops of the same round: children that pass the round's
    // selection test propagate at once, against the same snapshot, up to
    // `hops` propagations per round. Distances do not depend on the order in
    // which windows propagate; stale snapshot values only prune less.
    for (int32_t h = 1; h < hops; ++h) {
      hop_in.clear();
      std::vector<Cand> stay;
      for (const Cand& c : kids) (selected(c.key) ? hop_in : stay).push_back(c);
      kids.swap(stay);
      if (hop_in.empty()) break;
      for (const Cand& c : hop_in) {
        nsel++;
        propagate(M, c.b0, c.b1, c.px, c.py, c.sg, c.e, c.src, g.data(), AD.data(), AX.data(), ch_on, ich_on, retest,
                  eps_tiny, dev, aev, kids, C);
      }
    }
    add(nextp, kids);
    const int64_t ndev_prop = (int64_t)dev.size();
    for (const Ev& x : pending) dev.push_back(x);
    pending.clear();
    // Algorithm 4: the smallest value per key wins
    for (const Ev& x : dev) {
      if (x.d < g[x.v]) {
        g[x.v] = x.d;
      }
    }
    for (const AEv& a : aev) {
      if (a.D < AD[a.e] || (a.D == AD[a.e] && a.X < AX[a.e])) {
        AD[a.e] = a.D;
        AX[a.e] = a.X;
      }
    }
    ang_updates += (int64_t)aev.size();
    // One fan per pseudo-source vertex whose distance this round's events
    // lowered: among the winning events (d equal to the new geod_dist) the one
    // with the smallest incoming angle. Arrivals with equal distance from other
    // directions need no fan of their own: a direction outside the chosen
    // sector bends by less than pi against the chosen arrival, so a shorter
    // path exists.
    fw.clear();
    int64_t nfans = 0;
    touched.clear();
    for (const Ev& x : dev) {
      if (x.d != g[x.v]) continue;
      if (fan_th[x.v] == INFINITY) touched.push_back(x.v);
      if (x.th < fan_th[x.v]) fan_th[x.v] = x.th;
    }
    for (int32_t v : touched) {
      updates++;
      if (vupd) vupd[v]++;
      if (M.pseudo[v]) {
        fan(M, v, g[v], fan_th[v], full_fan, g.data(), eps_tiny, ich_on, fw, pending, C);
        nfans++;
      }
      fan_th[v] = INFINITY;
    }
    add(nextp, fw);
    if (rlog && rounds < max_log) {
      int64_t* r = rlog + rounds * RL_WIDTH;
      r[RL_N] = N;
      r[RL_CUTBITS] = (ext || dmode) ? (int64_t)bits_of(cval) : (cut.all ? -1 : (int64_t)cut.T);
      r[RL_SHIFT] = ext ? -2 : (dmode ? -3 : cut.shift);
      r[RL_SEL] = nsel;
      r[RL_STALE] = nstale;
      r[RL_KIDS] = C.kept;
      r[RL_TINY] = C.tiny;
      r[RL_ICH] = C.ich;
      r[RL_DEV] = ndev_prop;
      r[RL_AEV] = (int64_t)aev.size();
      r[RL_FANS] = nfans;
      r[RL_FANWIN] = C.fan_kept;
      r[RL_DEFER] = (int64_t)pending.size();
      r[RL_NEND] = (int64_t)nextp.size();
    }
    if (dmode) {
      double ratio = (double)k / (double)(nsel > 0 ? nsel : 1);
      double f = ratio < 0.5 ? 0.5 : (ratio > 2.0 ? 2.0 : ratio);
      delta = delta * f;
    }
    processed += nsel;
    stale_tot += nstale;
    Ctot.tiny += C.tiny;
    Ctot.ich += C.ich;
    Ctot.fans += C.fans;
    Ctot.fan_kept += C.fan_kept;
    Ctot.notwin += C.notwin;
    Ctot.deferred += C.deferred;
    pool.swap(nextp);
    rounds++;
  }
  for (int64_t v = 0; v < M.nv; ++v) dist[v] = g[v];
  if (n_rounds) *n_rounds = rounds;
  if (stats) {
    int64_t s[16] = {created, processed, stale_tot, Ctot.tiny, Ctot.ich, updates, ang_updates, Ctot.fans,
                     Ctot.fan_kept, rounds, peak, Ctot.notwin, Ctot.deferred, 0, 0, 0};
    std::memcpy(stats, s, sizeof(s));
  }
  return OK;
}

}  // namespace

// --------------------------------------------------------------------------
// C entry points (ctypes)
// --------------------------------------------------------------------------
extern "C" {

int orc_replica(const int32_t* faces, int64_t nf, int64_t nv, const double* he_len, const int32_t* src, int32_t m,
                int64_t k, int32_t hops, double eps_tiny, int32_t filters, int32_t mode, double delta0,
                const double* cut_table,
                int64_t n_cut, double* dist, int64_t* stats, int64_t* rlog, int64_t max_log, int64_t* n_rounds,
                int64_t* vupd) {
  OMesh M;
  int rc = build_mesh(faces, nf, nv, he_len, M);
  if (rc) return rc;
  std::vector<int32_t> s;
  rc = sorted_sources(src, m, nv, s);
  if (rc) return rc;
  if (k < 1) return fail(EINVAL_, "k must be >= 1");
  if (hops < 1) return fail(EINVAL_, "hops must be >= 1");
  if (mode != 0 && mode != 1) return fail(EINVAL_, "unknown selection mode");
  if (mode == 1 && !(delta0 > 0.0)) return fail(EINVAL_, "delta0 must be > 0");
  return run_replica(M, s.data(), (int32_t)s.size(), k, hops, eps_tiny, filters, mode, delta0, cut_table, n_cut,
                     dist, stats, rlog, max_log, n_rounds, vupd);
}

// Own elementary functions, exported so tests can check them against libm.
double orc_fn_atan2(double y, double x) { return orc_atan2(y, x); }
void orc_fn_sincos(double t, double* s, double* c) { orc_sincos(t, s, c); }

}  // extern "C"
