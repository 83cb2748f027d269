// PCH round pipeline on gfx950: device kernels, the host round driver and the
// C ABI of include/pch.h.
//
// One round (Section 4.2, Algorithm 1) is a fixed sequence of kernels on one
// stream; counts live in device memory, so rounds are enqueued back to back
// and the host only polls a control block every few rounds:
//   hist/scan  - three 12-bit histogram passes give the k-th smallest key
//                (selection, step 1; only for the k-th-key rule)
//   partition  - drop stale windows, split the pool into selected windows and
//                survivors (the gap-free pool of Section 4.1 and Algorithm 3)
//   org        - optional: group the selected windows by edge
//   propagate  - Algorithm 2 for every selected window against the round-start
//                state, once per hop (children that pass the round's selection
//                test propagate again in the same round); children and events
//                are appended with one reservation per wavefront (Algorithm 3's
//                prefix sum, done per wave)
//   events 1-3 - Algorithm 4: per-vertex minimum of distance events and
//                per-corner lexicographic minimum of angle events, the
//                incoming angles of the winning events, then one fan of
//                windows per improved pseudo-source vertex (Figure 3(c)); the
//                last workgroup of the third pass closes the round's log
//                record and sets up the next round's selection
// The batched form runs the same phases for one field per workgroup inside a
// persistent kernel, separated by workgroup barriers.
//
// All window geometry is FP64; the file is compiled with FP contraction off so
// results do not depend on instruction selection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdio>
#include <string>
#include <vector>

#include "pch.h"
#include "pch_internal.h"

using u64 = unsigned long long;
using u32 = unsigned int;

namespace {

thread_local std::string t_err;

pch_status set_err(pch_status s, const std::string& m) {
  t_err = m;
  return s;
}

constexpr int kCdfBins = 65536;
constexpr int kMaxHops = 16;  // propagation hops per round at most
constexpr int kOrgBuckets = 4096;  // edge buckets of the organization by edge

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return set_err(e_ == hipErrorOutOfMemory ? PCH_ENOMEM : PCH_EDEVICE,              \
                     std::string(#expr) + ": " + hipGetErrorString(e_));                \
  } while (0)

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kHistBins = 4096;
constexpr int kSmallGrid = 128;
constexpr u64 kAllOnes = ~0ull;
constexpr int64_t kMaxRounds = 1 << 24;
// the no-alloc entry point: its work buffers live in `scratch` (below)
constexpr int kNoallocMaxSources = 1024;
constexpr size_t kScratchBytes = (size_t)256 << 20;

// constants of the window arithmetic (same values as the method description)
constexpr double kTau = 1e-12;             // endpoint / occupancy tolerance, relative to L
constexpr double kEv = 1.0 - 1e-12;        // event raised when d < g * kEv
// Filters drop a window only when the dominating path is shorter by more than
// a relative 1e-12, so near-ties are never decided by rounding (a window that
// grazes a nearly straight convex boundary vertex can be the only one carrying
// rays past it).
constexpr double kFm = 1.0 + 1e-12;
constexpr double kPi = 3.14159265358979323846;
constexpr double kHalfPi = 0.5 * 3.14159265358979323846;
constexpr double kQuarterPi = 0.25 * 3.14159265358979323846;

// per-round counters (also the per-round log record layout, see pch.h)
enum {
  C_N = 0, C_CUT, C_SHIFT, C_SEL, C_STALE, C_KIDS, C_TINY, C_ICH, C_DEV, C_AEV, C_FANS, C_FANWIN, C_DEFER,
  C_NEND, C_NUM
};
// extra counters (not in the log)
enum { X_NOTWIN = 0, X_SEL1 = 1, X_NUM = 4 };  // X_SEL1: windows the pool scans selected (hop 1)

// A pair of counters indexed by parity, each alone in its 128-byte line.
// Atomics that fall in the same 64-byte granule of memory are performed one
// after another (about 12.5 ns apiece on gfx950, measured with one returning
// atomicAdd per workgroup: one counter, or four 8 bytes apart, 80 M/s; four
// 128 bytes apart, 280 M/s), so every counter that the workgroups of one
// launch update with atomics gets a line of its own.
struct Pair {
  u64 d[2][16];
  __host__ __device__ u64& operator[](u64 i) { return d[i][0]; }
  __host__ __device__ const u64& operator[](u64 i) const { return d[i][0]; }
};

struct Ctl {
  // updated with atomics by the workgroups of a launch
  Pair npool;                // slots used in pool buffer 0 and 1 (live windows and tombstones)
  Pair ndev;                 // distance events recorded for the round of each parity
  Pair kmin, kmax;           // key range of the next pool, by parity
  alignas(128) u64 naev;     // angle events of the current round
  alignas(128) u64 ncand;    // fan candidates of the current round
  alignas(128) u64 keptin;   // windows the pool scan kept in place
  alignas(128) u64 ticket;   // last-block detection
  alignas(128) u64 nsel;
  alignas(128) u64 scan_next;  // next free ticket of the fused pool scan
  alignas(128) u64 cnt[C_NUM];  // current round
  alignas(128) u64 xcnt[X_NUM];
  alignas(128) u64 nhop[kMaxHops + 1];  // nhop[h]: windows queued by hop h for hop h + 1
  alignas(128) u64 overflow;  // rare flags
  u64 nonfinite;
  u64 badidx;       // a window or event named a half-edge or vertex outside the mesh
  // set by the round set-up, read by the launches
  alignas(128) u64 round;  // rounds run so far
  u64 active;       // 1 while the current round has work
  u64 done;
  u64 sel_all;      // current round selects every window
  u64 shift;        // key bits dropped before comparing
  u64 want;         // selected truncated-key prefix after the histogram passes
  u64 rank;         // remaining rank inside the current histogram bin
  u64 use_table;    // current round selects key <= cutval
  double cutval;
  u64 dmode;        // current round uses the adaptive step
  double delta;     // adaptive step
  u64 lmode;        // current round uses the learned cutoff
  double lfac;      // feedback factor of the learned cutoff
  u64 tot[C_NUM];   // totals over all rounds
  u64 peak;
  u64 smode;        // current round uses the strided selection
  // The pool: the round's windows are the live slots [0, nscan) of buffer
  // pin. The partition either leaves the windows it keeps in place (selected
  // and stale ones become tombstones) and the round appends its new windows
  // to the same buffer after slot s0 = nscan, or it compacts the kept windows
  // into the other buffer (s0 = 0); pout is the buffer that receives them.
  // The next round's live windows are keptin (kept in place) plus the slots
  // appended after s0.
  u64 pin, pout, nscan, s0;
};
static_assert(sizeof(Ctl) % 128 == 0, "control block is whole 128-byte lines");

// key of a tombstone: a pool slot whose window was selected or dropped (no
// finite non-negative key has this bit pattern, and no histogram prefix of
// one matches it)
constexpr u64 kDead = ~0ull;

// A pool of windows (Section 3, Figure 2): the interval [b0, b1] of
// half-edge e, the pseudo-source (px, py) in e's frame, its distance sg from
// the source, the selection key and the pseudo-source vertex src, stored as
// four arrays of pairs so that a wavefront moves each pair with one fully
// coalesced 16-byte (8-byte for (e, src)) access per lane.
struct Pool {
  double2* bb;  // (b0, b1)
  double2* pp;  // (px, py)
  double2* sk;  // (sg, key)
  int2* es;     // (e, src)
};

// Distance events: vertex v reached at distance d, and the incoming angle a
// fan at a pseudo-source needs. An event from propagation stores how to get
// the angle, q = 4 e + k for vertex k of half-edge e and (x, y) the window's
// pseudo-source in e's frame; the second event pass evaluates it for the
// events that win their vertex and stores it back as q = -1, x = angle.
struct DistEv {
  int2* vq;     // (v, q)
  double* d;
  double2* xy;
};

struct AngEv {
  int32_t* e;
  double *D, *X;
};

// The half-edge record and its constants share one 128-byte cache line, so a
// window's propagation gathers one line for its half-edge.
struct alignas(128) HalfEdgeLine {
  pch::HalfEdge h;
  pch::HalfEdgeAng a;
};
static_assert(sizeof(HalfEdgeLine) == 128, "half-edge line must be 128 bytes");

// angle_split of one corner (oriented edge): the best apex distance (bit
// pattern) and its crossing (order-preserving key), side by side in 16 bytes.
struct alignas(16) Split {
  u64 D, X;
};

struct DevMesh {
  const HalfEdgeLine* hl;
  const double* phi;
  const double* alpha;
  const int32_t* twin;
  const int32_t* hv;
  const double* theta;
  const uint8_t* flags;
  const int32_t* coff;
  const int32_t* corner;
  const pch::Corner* crec;
  int32_t nv, nh;  // vertices and half-edges: every gathered index is checked against them
};

// geod_dist and angle_split are kept twice. The round reads g and as, the
// values at its start (the delayed update of Remark 3), while the events it
// raises lower gw and asw at once; the event passes then copy the values
// that changed back into g and as, so that both pairs agree again when the
// next round starts.
struct DevState {
  u64* g;      // geod_dist as bit patterns (non-negative doubles order as u64)
  Split* as;   // angle_split per oriented edge
  u64* fanth;  // smallest incoming angle key among this round's winning events
  u32* claim;  // round stamp of the last fan expanded at a vertex
  u64* gw;     // geod_dist taking this round's minima
  Split* asw;  // angle_split taking this round's minima
};

struct RoundArgs {
  DevMesh m;
  DevState s;
  Pool pool[2];
  Pool sel;
  Pool hq[2];      // hop queues: hop h reads hq[h & 1] (h >= 2), writes hq[(h + 1) & 1]
  DistEv ev[2];
  DistEv cand;     // the round's events that won a pseudo-source vertex: (v, d, angle)
  AngEv aev;
  Ctl* ctl;
  u32* hist;
  int64_t* log;    // [max_log][C_NUM] or null
  int64_t max_log;
  int64_t cap;     // windows per pool buffer
  int64_t ecap;    // distance events per buffer
  int64_t acap;    // angle events
  int64_t k;
  int32_t mode;
  double eps;
  int32_t ch_on, ich_on, full_fan, retest;
  const double* table;  // device cutoff table or null
  int64_t n_table;
  const u32* cdf;       // learned cutoff: cumulative counts of predicted distances
  double pbin;          // width of a cdf bin
  double w0;            // windows per vertex before the first learned round
  int32_t hops;         // propagation hops per round (1 = each selected window once)
  int32_t counts;       // 1 = count windows, events and drops (statistics only)
  // organization by edge: the selected windows are grouped by the bucket
  // e >> org_shift of their half-edge before they propagate (org_shift < 0: off)
  int32_t org_shift;
  Pool sorted;
  u32* org_hist;  // [kOrgBuckets] selected windows per bucket
  u32* org_ofs;   // [kOrgBuckets] next free slot per bucket
};

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ u64 bits(double x) { return (u64)__double_as_longlong(x); }
__device__ __forceinline__ double from_bits(u64 u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ u64 ordkey(double x) {
  const u64 u = bits(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordkey(u64 k) {
  return (k >> 63) ? from_bits(k & 0x7fffffffffffffffull) : from_bits(~k);
}
// Reads of geod_dist, angle_split and the fan keys, which are updated with
// device-scope atomics (performed in L2): agent-scope loads bypass stale
// vector-L1 lines, so phases of one workgroup see each other's updates
// without invalidating the whole L1.
__device__ __forceinline__ u64 lda(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int he_next(int j) { return j - j % 3 + (j % 3 + 1) % 3; }
__device__ __forceinline__ int he_prev(int j) { return j - j % 3 + (j % 3 + 2) % 3; }
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ u64 shfl64(u64 x, int src) {
  u32 lo = __shfl((u32)x, src, kWave);
  u32 hi = __shfl((u32)(x >> 32), src, kWave);
  return ((u64)hi << 32) | lo;
}

// Up to four reservations from one prefix sum: the last lane issues the
// atomics back to back so that their round trips overlap. Every per-lane
// count is at most 3, so the four counts travel packed in the bytes of one
// 32-bit word (a wavefront's totals stay below 256). Every lane of the
// wavefront must call it; counters with a zero total get no atomic.
__device__ __forceinline__ void wave_reserve4(u64* c0, u32 n0, u64* c1, u32 n1, u64* c2, u32 n2, u64* c3, u32 n3,
                                              u64& s0, u64& s1, u64& s2, u64& s3, u32& t0, u32& t1, u32& t2,
                                              u32& t3) {
  const int lane = lane_id();
  const u32 x = n0 | (n1 << 8) | (n2 << 16) | (n3 << 24);
  u32 incl = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const u32 y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  const u32 tot = __shfl(incl, kWave - 1, kWave);
  const u32 excl = incl - x;
  t0 = tot & 0xffu;
  t1 = (tot >> 8) & 0xffu;
  t2 = (tot >> 16) & 0xffu;
  t3 = tot >> 24;
  u64 b0 = 0, b1 = 0, b2 = 0, b3 = 0;
  if (lane == kWave - 1) {
    if (t0) b0 = atomicAdd(c0, (u64)t0);
    if (t1) b1 = atomicAdd(c1, (u64)t1);
    if (t2) b2 = atomicAdd(c2, (u64)t2);
    if (t3) b3 = atomicAdd(c3, (u64)t3);
  }
  s0 = shfl64(b0, kWave - 1) + (excl & 0xffu);
  s1 = shfl64(b1, kWave - 1) + ((excl >> 8) & 0xffu);
  s2 = shfl64(b2, kWave - 1) + ((excl >> 16) & 0xffu);
  s3 = shfl64(b3, kWave - 1) + (excl >> 24);
}

// The four reservations of wave_reserve4 for a whole workgroup: one atomic
// per counter and workgroup instead of one per wavefront, so 4x fewer
// same-address atomics meet at the counters. Every thread of the workgroup
// must call it (it holds two barriers); a counter may be in LDS. BS is the
// workgroup size.
template <int BS = kBlock>
__device__ __forceinline__ void block_reserve4(u64* c0, u32 n0, u64* c1, u32 n1, u64* c2, u32 n2, u64* c3, u32 n3,
                                               u64& s0, u64& s1, u64& s2, u64& s3, u32& t0, u32& t1, u32& t2,
                                               u32& t3) {
  constexpr int kW = BS / kWave;
  __shared__ u32 s_w[kW][4];  // wavefront totals
  __shared__ u64 s_b[kW][4];  // wavefront bases
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const u32 x = n0 | (n1 << 8) | (n2 << 16) | (n3 << 24);
  u32 incl = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const u32 y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  const u32 tot = __shfl(incl, kWave - 1, kWave);
  const u32 excl = incl - x;
  t0 = tot & 0xffu;
  t1 = (tot >> 8) & 0xffu;
  t2 = (tot >> 16) & 0xffu;
  t3 = tot >> 24;
  if (lane == kWave - 1) {
    s_w[w][0] = t0;
    s_w[w][1] = t1;
    s_w[w][2] = t2;
    s_w[w][3] = t3;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int j = threadIdx.x;
    u64* cj = j == 0 ? c0 : j == 1 ? c1 : j == 2 ? c2 : c3;
    u32 sum = 0;
#pragma unroll
    for (int q = 0; q < kW; ++q) sum += s_w[q][j];
    u64 base = sum ? atomicAdd(cj, (u64)sum) : 0;
#pragma unroll
    for (int q = 0; q < kW; ++q) {
      s_b[q][j] = base;
      base += s_w[q][j];
    }
  }
  __syncthreads();
  s0 = s_b[w][0] + (excl & 0xffu);
  s1 = s_b[w][1] + ((excl >> 8) & 0xffu);
  s2 = s_b[w][2] + ((excl >> 16) & 0xffu);
  s3 = s_b[w][3] + (excl >> 24);
}

// Three reservations (per-lane counts at most 3), as wave_reserve4.
__device__ __forceinline__ void wave_reserve3(u64* c0, u32 n0, u64* c1, u32 n1, u64* c2, u32 n2, u64& s0, u64& s1,
                                              u64& s2, u32& t0, u32& t1, u32& t2) {
  u64 s3;
  u32 t3;
  wave_reserve4(c0, n0, c1, n1, c2, n2, c0, 0u, s0, s1, s2, s3, t0, t1, t2, t3);
}

__device__ __forceinline__ u32 wave_sum(u32 x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

__device__ __forceinline__ u64 wave_min64(u64 x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    u64 y = shfl64(x, lane_id() ^ o);
    x = y < x ? y : x;
  }
  return x;
}
__device__ __forceinline__ u64 wave_max64(u64 x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    u64 y = shfl64(x, lane_id() ^ o);
    x = y > x ? y : x;
  }
  return x;
}

// atan on [0, 1]: two half-angle reductions atan(t) = 2 atan(t / (1 + sqrt(1 + t^2)))
// bring the argument below tan(pi/16); then 13 terms of the Maclaurin series
// (Horner in u^2). Uses only + - * / sqrt, so it rounds the same everywhere.
__device__ double dev_atan01(double t) {
  double u = t / (1.0 + sqrt(1.0 + t * t));
  u = u / (1.0 + sqrt(1.0 + u * u));
  const double u2 = u * u;
  double p = 0.0;
  // unrolled: the coefficients 1/(2i+1) fold to correctly rounded constants
#pragma unroll
  for (int i = 12; i >= 0; --i) {
    double c = 1.0 / (double)(2 * i + 1);
    if (i & 1) c = -c;
    p = p * u2 + c;
  }
  return 4.0 * (u * p);
}

__device__ double dev_atan2(double y, double x) {
  const double ax = fabs(x), ay = fabs(y);
  if (ax == 0.0 && ay == 0.0) return 0.0;
  double r = ay > ax ? kHalfPi - dev_atan01(ax / ay) : dev_atan01(ay / ax);
  if (x < 0.0) r = kPi - r;
  if (y < 0.0) r = -r;
  return r;
}

// sin/cos on [0, pi/4] from 11 nested Maclaurin factors; [0, pi] folded by
// symmetry.
__device__ void dev_sincos_small(double u, double* s, double* c) {
  const double u2 = u * u;
  double ps = 1.0, pc = 1.0;
  // unrolled: the reciprocals 1/((2n)(2n+1)) and 1/((2n-1)(2n)) fold to
  // correctly rounded constants
#pragma unroll
  for (int n = 11; n >= 1; --n) {
    const double rs = 1.0 / ((double)(2 * n) * (double)(2 * n + 1));
    const double rc = 1.0 / ((double)(2 * n - 1) * (double)(2 * n));
    ps = 1.0 - (u2 * rs) * ps;
    pc = 1.0 - (u2 * rc) * pc;
  }
  *s = u * ps;
  *c = pc;
}

__device__ void dev_sincos(double t, double* s, double* c) {
  double sc = 1.0;
  if (t > kHalfPi) {
    t = kPi - t;
    sc = -1.0;
  }
  double ss, cc;
  if (t > kQuarterPi)
    dev_sincos_small(kHalfPi - t, &cc, &ss);
  else
    dev_sincos_small(t, &ss, &cc);
  *s = ss;
  *c = sc * cc;
}



// Selection key: distance from the source to the nearest point of the window
// (the pseudo-source's distance plus its distance to the interval). The key
// and the child filter below take their square roots before any decision
// (straight-line code, so that independent roots overlap).
__device__ __forceinline__ double window_key(double b0, double b1, double px, double py, double sg) {
  const double dx = px < b0 ? b0 - px : px - b1;
  const double dseg = sqrt(dx * dx + py * py);
  return sg + ((px < b0 || px > b1) ? dseg : -py);
}

// Tiny-window trim and the Xin-Wang filter of Figure 4(b). u0/u1 are the
// start/end vertices of the child's edge; the third test (vertex r of the
// face just crossed) is made at the endpoint next to the shared vertex.
// Returns 0 keep, 1 tiny, 2 filtered.
__device__ __forceinline__ int child_filter(double c0, double c1, double cpx, double cpy, double sg, double lc,
                                            double gu0, double gu1, bool rtest, bool r_at_c0, double gr,
                                            double rdist, double eps, bool ich_on) {
  const double dx1 = c1 - cpx;
  const double f1 = sg + sqrt(dx1 * dx1 + cpy * cpy);
  const double dx0 = c0 - cpx;
  const double f0 = sg + sqrt(dx0 * dx0 + cpy * cpy);
  if (!(c1 - c0 > eps * lc)) return 1;
  if (!ich_on) return 0;
  if (f1 > (gu0 + c1) * kFm) return 2;
  if (f0 > (gu1 + (lc - c0)) * kFm) return 2;
  if (rtest && (r_at_c0 ? f0 : f1) > (gr + rdist) * kFm) return 2;
  return 0;
}

__device__ __forceinline__ void store_window(const Pool& P, u64 i, double b0, double b1, double px, double py,
                                             double sg, double key, int32_t e, int32_t src) {
  P.bb[i] = make_double2(b0, b1);
  P.pp[i] = make_double2(px, py);
  P.sk[i] = make_double2(sg, key);
  P.es[i] = make_int2(e, src);
}

// A list of hop windows in LDS: like a pool without the key, which the
// propagation of a window does not read (48 bytes per window).
struct HopList {
  double2* bb;
  double2* pp;
  double* sg;
  int2* es;
};

__device__ __forceinline__ void store_window(const HopList& P, u64 i, double b0, double b1, double px, double py,
                                             double sg, double, int32_t e, int32_t src) {
  P.bb[i] = make_double2(b0, b1);
  P.pp[i] = make_double2(px, py);
  P.sg[i] = sg;
  P.es[i] = make_int2(e, src);
}

__device__ __forceinline__ void flag_overflow(Ctl* c) { atomicOr(&c->overflow, 1ull); }

// Range guard of a gathered index (a window's half-edge or pseudo-source, an
// event's vertex or corner): an index outside [0, n) is never dereferenced; it
// sets the control block's badidx flag, and the host reports an error for the
// field instead of reading outside the mesh's tables.
__device__ __forceinline__ bool idx_ok(Ctl* c, int32_t i, int32_t n) {
  if ((u32)i < (u32)n) return true;
  atomicOr(&c->badidx, 1ull);
  return false;
}

// Incoming angle of a propagation event (q = 4 e + k, pseudo-source (px, py)
// in e's frame): the angular position around vertex k of half-edge e of the
// direction back towards the pseudo-source.
__device__ __forceinline__ double event_angle(const DevMesh& m, int q, double px, double py) {
  const int e = q >> 2, k = q & 3;
  const pch::HalfEdge h = m.hl[e].h;
  const pch::HalfEdgeAng ha = m.hl[e].a;
  if (k == 0) return ha.th0 - dev_atan2(-py, px);
  if (k == 1) return ha.th1 + dev_atan2(-py, h.L - px);
  const double x2 = h.x2, y2 = h.y2;
  const double ux = -x2, uy = -y2, wx = px - x2, wy = py - y2;
  const double cr = ux * wy - uy * wx;
  const double dt = ux * wx + uy * wy;
  return ha.th2 + dev_atan2(cr, dt);
}

// The half-edge values an incoming angle needs (loaded ahead of the decision
// to evaluate it), and the angle from them: the same arithmetic as
// event_angle.
struct AngleRecipe {
  double th, L, x2, y2;
  int k;
};
__device__ __forceinline__ AngleRecipe load_recipe(const DevMesh& m, int q) {
  const int e = q >> 2, k = q & 3;
  const pch::HalfEdge h = m.hl[e].h;
  const pch::HalfEdgeAng ha = m.hl[e].a;
  return AngleRecipe{k == 0 ? ha.th0 : (k == 1 ? ha.th1 : ha.th2), h.L, h.x2, h.y2, k};
}
__device__ __forceinline__ double recipe_angle(const AngleRecipe& r, double px, double py) {
  if (r.k == 0) return r.th - dev_atan2(-py, px);
  if (r.k == 1) return r.th + dev_atan2(-py, r.L - px);
  const double ux = -r.x2, uy = -r.y2, wx = px - r.x2, wy = py - r.y2;
  const double cr = ux * wy - uy * wx;
  const double dt = ux * wx + uy * wy;
  return r.th + dev_atan2(cr, dt);
}

// One corner of a fan of windows from pseudo-source vertex v reached at
// distance d, the incoming ray's back direction at angular position th
// (Figure 3(c)). A corner that meets the sector of directions at least pi away
// from th on both sides (all directions when full) yields a window on the far
// side of its opposite edge, clipped to the sector, and distance events for its
// endpoints that lie in the sector (the straight edge path).
struct FanOut {
  bool win;
  double b0, b1, px, py, key;
  int32_t e;
  bool ea, eb;  // distance events at the corner's vertices a and b
  int32_t va, vb;
  double da, db, tha, thb;
};

__device__ void fan_corner(const RoundArgs& a, int v, double d, double th, bool full, int q, FanOut& o,
                           u32& tiny, u32& ich, u32& notwin) {
  o.win = false;
  o.ea = o.eb = false;
  const DevMesh& m = a.m;
  const u64* g = a.s.g;
  const pch::Corner cr = m.crec[q];
  const double al = cr.alpha;
  double t0, t1;
  if (full) {
    t0 = 0.0;
    t1 = al;
  } else if (!(m.flags[v] & pch::VF_BOUNDARY)) {
    const double Th = m.theta[v];
    double rel = cr.phi - th;
    if (!isfinite(rel)) return;
    while (rel < 0.0) rel += Th;
    while (rel >= Th) rel -= Th;
    const double lo = kPi - rel;
    const double hi = (Th - kPi) - rel;
    t0 = lo > 0.0 ? lo : 0.0;
    t1 = hi < al ? hi : al;
    if (!(t0 <= t1)) return;
  } else {
    const double rel = cr.phi - th;
    const double hiA = -kPi - rel;
    const double loB = kPi - rel;
    if (hiA >= 0.0) {
      t0 = 0.0;
      t1 = hiA < al ? hiA : al;
    } else if (loB <= al) {
      t0 = loB > 0.0 ? loB : 0.0;
      t1 = al;
    } else {
      return;
    }
  }
  const int va = cr.a;
  const int vb = cr.b;
  const double ga = from_bits(lda(&g[va])), gb = from_bits(lda(&g[vb]));
  if (t0 <= 0.0) {
    const double da = d + cr.l_va;
    if (da < ga * kEv) {
      o.ea = true;
      o.va = va;
      o.da = da;
      o.tha = cr.th_a;
    }
  }
  if (t1 >= al && cr.last) {
    const double db = d + cr.l_vb;
    if (db < gb * kEv) {
      o.eb = true;
      o.vb = vb;
      o.db = db;
      o.thb = cr.th_b;
    }
  }
  const int tw = cr.tw;
  if (tw < 0) {
    notwin++;
    return;
  }
  const double Ln = cr.L, x2n = cr.x2, y2n = cr.y2;
  const double ipx = Ln - x2n, ipy = -y2n;
  double c0, c1;
  if (t1 >= al) {
    c0 = 0.0;
  } else {
    double sn, cs;
    dev_sincos(t1, &sn, &cs);
    const double dx = cs * x2n - sn * y2n, dy = sn * x2n + cs * y2n;
    c0 = ipx - ipy * (dx / dy);
  }
  if (t0 <= 0.0) {
    c1 = Ln;
  } else {
    double sn, cs;
    dev_sincos(t0, &sn, &cs);
    const double dx = cs * x2n - sn * y2n, dy = sn * x2n + cs * y2n;
    c1 = ipx - ipy * (dx / dy);
  }
  if (c0 < 0.0) c0 = 0.0;
  if (c1 > Ln) c1 = Ln;
  const int r = child_filter(c0, c1, ipx, ipy, d, Ln, gb, ga, false, false, 0.0, 0.0, a.eps, a.ich_on);
  if (r == 1) {
    tiny++;
    return;
  }
  if (r == 2) {
    ich++;
    return;
  }
  o.win = true;
  o.b0 = c0;
  o.b1 = c1;
  o.px = ipx;
  o.py = ipy;
  o.key = window_key(c0, c1, ipx, ipy, d);
  o.e = tw;
}

__device__ __forceinline__ int wave_max_i(int x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const int y = __shfl_xor(x, o, kWave);
    x = y > x ? y : x;
  }
  return x;
}

__device__ __forceinline__ double shfl_d(double x, int src) {
  return from_bits(shfl64(bits(x), src));
}

// Fans of the lanes of one wavefront (has = this lane expands a fan of vertex
// v at distance d). The wavefront's (fan, corner) pairs are spread over its
// lanes: an exclusive prefix sum of the fan degrees numbers the pairs and each
// lane finds the owner of its pair by binary search over the lanes. Windows
// and events are reserved once per wavefront and step (kBlk: once per
// workgroup and step, every thread of the workgroup calling it, so that a
// launch's waves meet at the two counters 4x less often); windows go to pool
// buffer po, events to event buffer qi. Every lane of the wavefront must call
// it.
// The lane's corners are q0 .. q0 + deg - 1 of the CCW corner list (deg = 0
// when it has no fan).
template <bool kBlk = false>
__device__ void wave_fans(const RoundArgs& a, bool has, int v, int q0, int deg, double d, double th, bool full,
                          int po, int qi, u64& kmn, u64& kmx, u32& kept, u32& tiny, u32& ich, u32& defer,
                          u32& notwin) {
  Ctl* c = a.ctl;
  const int lane = lane_id();
  if (!has) deg = 0;
  int incl = deg;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  const int total = __shfl(incl, kWave - 1, kWave);
  const int base = incl - deg;
  const Pool P = po ? a.pool[1] : a.pool[0];
  const DistEv& E = a.ev[qi];
  for (int t0 = 0; kBlk ? __syncthreads_or(t0 < total) : t0 < total; t0 += kWave) {
    const int t = t0 + lane;
    // owner: the largest lane whose base is <= t (lanes with deg 0 share the
    // base of the next lane, so the largest such lane owns the pair)
    int lo = 0, hi = kWave - 1;
#pragma unroll
    for (int it = 0; it < 6; ++it) {
      const int mid = (lo + hi + 1) >> 1;
      const int bm = __shfl(base, mid, kWave);
      if (bm <= t) lo = mid; else hi = mid - 1;
    }
    const int owner = lo;
    const int ov = __shfl(v, owner, kWave);
    const int oq = __shfl(q0, owner, kWave) + (t - __shfl(base, owner, kWave));
    const double od = shfl_d(d, owner);
    const double oth = shfl_d(th, owner);
    FanOut o;
    o.win = false;
    o.ea = o.eb = false;
    if (t < total) fan_corner(a, ov, od, oth, full, oq, o, tiny, ich, notwin);
    const u32 nev = (o.ea ? 1u : 0u) + (o.eb ? 1u : 0u);
    u64 jw, je, jz;
    u32 tw, te, tz;
    if constexpr (kBlk) {
      u64 j3;
      u32 t3;
      block_reserve4(&c->npool[po], o.win ? 1u : 0u, &c->ndev[qi], nev, &c->ndev[qi], 0u, &c->ndev[qi], 0u, jw, je,
                     jz, j3, tw, te, tz, t3);
    } else {
      wave_reserve3(&c->npool[po], o.win ? 1u : 0u, &c->ndev[qi], nev, &c->ndev[qi], 0u, jw, je, jz, tw, te, tz);
    }
    if (o.win) {
      if (jw < (u64)a.cap) {
        store_window(P, jw, o.b0, o.b1, o.px, o.py, od, o.key, o.e, ov);
        const u64 kb = bits(o.key);
        kmn = kb < kmn ? kb : kmn;
        kmx = kb > kmx ? kb : kmx;
      } else {
        flag_overflow(c);
      }
      kept++;
    }
    // deferred events lower geod_dist's write copy now; they are recorded in
    // the next round's event buffer, whose passes copy the winners back
    if (o.ea) atomicMin(&a.s.gw[o.va], bits(o.da));
    if (o.eb) atomicMin(&a.s.gw[o.vb], bits(o.db));
    if (o.ea) {
      if (je < (u64)a.ecap) {
        E.vq[je] = make_int2(o.va, -1);
        E.d[je] = o.da;
        E.xy[je] = make_double2(o.tha, 0.0);
      } else {
        flag_overflow(c);
      }
      je++;
    }
    if (o.eb) {
      if (je < (u64)a.ecap) {
        E.vq[je] = make_int2(o.vb, -1);
        E.d[je] = o.db;
        E.xy[je] = make_double2(o.thb, 0.0);
      } else {
        flag_overflow(c);
      }
    }
    defer += nev;
  }
}

// Workgroup totals of per-wave partial results, so that a phase issues one
// atomic per workgroup and counter instead of one per wavefront (same-address
// atomics serialize). Every thread of the workgroup must call it; the totals
// are valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_totals(u64& kmn, u64& kmx, u32 (&v)[NV]) {
  __shared__ u64 s_mn[16], s_mx[16];
  __shared__ u32 s_v[NV][16];
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  kmn = wave_min64(kmn);
  kmx = wave_max64(kmx);
#pragma unroll
  for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
  if (lane_id() == 0) {
    s_mn[w] = kmn;
    s_mx[w] = kmx;
#pragma unroll
    for (int j = 0; j < NV; ++j) s_v[j][w] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < nw; ++q) {
      kmn = s_mn[q] < kmn ? s_mn[q] : kmn;
      kmx = s_mx[q] > kmx ? s_mx[q] : kmx;
#pragma unroll
      for (int j = 0; j < NV; ++j) v[j] += s_v[j][q];
    }
  }
  __syncthreads();
}

// relaxed agent-scope load of a counter that other workgroups update atomically
__device__ __forceinline__ u64 ld(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lane 0's part of the round set-up for input parity p: log and total the
// previous round, stop when nothing is left, reset this round's output buffers
// and set up the selection rule. Every counter it reads is loaded first, in one
// batch of independent loads, so the set-up costs a few memory round trips.
// Returns 1 when the round takes the learned cutoff: *want is then the number
// of vertices whose predicted distance the cutoff must reach and *m the pool's
// smallest key.
__device__ int round_begin_lane0(const RoundArgs& a, int p, u64* want_out, double* m_out) {
  Ctl* c = a.ctl;
  const u64 done = ld(&c->done), active = ld(&c->active), overflow = ld(&c->overflow) | ld(&c->badidx);
  const u64 round = ld(&c->round), peak = ld(&c->peak);
  const u64 dmode = ld(&c->dmode), lmode = ld(&c->lmode);
  const u64 pout = ld(&c->pout), s0 = ld(&c->s0), keptin = ld(&c->keptin);
  const u64 slots = ld(&c->npool[pout & 1]), nd = ld(&c->ndev[p]);
  const u64 N = keptin + (slots - s0);  // live windows
  const u64 mn = ld(&c->kmin[p]), mx = ld(&c->kmax[p]);
  u64 rec[C_NUM], tot[C_NUM];
#pragma unroll
  for (int f = 0; f < C_NUM; ++f) rec[f] = ld(&c->cnt[f]);
#pragma unroll
  for (int f = 0; f < C_NUM; ++f) tot[f] = ld(&c->tot[f]);
  double delta = c->delta, lfac = c->lfac;
  if (done) return 0;
  if (active) {
    const u64 r = round - 1;
    rec[C_NEND] = N;
    rec[C_DEFER] = nd;
    const bool logit = a.log && (int64_t)r < a.max_log;
#pragma unroll
    for (int f = 0; f < C_NUM; ++f) {
      if (logit) a.log[r * C_NUM + f] = (int64_t)rec[f];
      tot[f] += rec[f];
      c->tot[f] = tot[f];
    }
    // adaptive step / learned feedback: steer the next cutoff toward k
    // selected windows
    if (dmode || lmode) {
      const u64 ns = rec[C_SEL];
      const double ratio = (double)a.k / (double)(ns > 0 ? ns : 1ull);
      const double f = ratio < 0.5 ? 0.5 : (ratio > 2.0 ? 2.0 : ratio);
      if (dmode) {
        delta = delta * f;
        c->delta = delta;
      } else {
        lfac = lfac * f;
        c->lfac = lfac;
      }
    }
    c->active = 0;
  }
  if (overflow || (N == 0 && nd == 0)) {
    c->done = 1;
    return 0;
  }
  c->active = 1;
  c->round = round + 1;
  if (N > peak) c->peak = N;
#pragma unroll
  for (int f = 0; f < C_NUM; ++f) c->cnt[f] = 0;
  c->cnt[C_N] = N;
  // the pool: keep the windows in place while at most half of the slots are
  // tombstones and at most a quarter of the buffer is used (the round
  // appends to the rest), else compact them into the other buffer
  c->pin = pout;
  c->nscan = slots;
  c->keptin = 0;
  if (slots - N > N || slots > (u64)a.cap / 4) {
    c->pout = pout ^ 1;
    c->npool[(pout ^ 1) & 1] = 0;
    c->s0 = 0;
  } else {
    c->s0 = slots;
  }
  c->ndev[1 - p] = 0;
  c->scan_next = 0;
  c->nsel = 0;
  c->naev = 0;
  c->ncand = 0;
  for (int h = 1; h < a.hops; ++h) c->nhop[h] = 0;
  c->kmin[1 - p] = kAllOnes;
  c->kmax[1 - p] = 0;
  c->use_table = 0;
  c->sel_all = 0;
  c->dmode = 0;
  c->lmode = 0;
  c->smode = 0;
  c->rank = 0;
  const u64 r = round;  // index of the round being set up
  if (a.table && (int64_t)r < a.n_table) {
    c->use_table = 1;
    c->cutval = a.table[r];
    c->cnt[C_CUT] = bits(c->cutval);
    c->cnt[C_SHIFT] = (u64)(int64_t)-2;
    return 0;
  }
  if (N <= (u64)a.k) {
    c->sel_all = 1;
    c->cnt[C_CUT] = (u64)(int64_t)-1;
    c->cnt[C_SHIFT] = 0;
    return 0;
  }
  if (a.mode == PCH_SELECT_LEARNED) {
    // C(m): vertices predicted within the pool's smallest key; w: windows
    // processed per such vertex so far (w0 before any)
    const double m = from_bits(mn);
    const double bm = m / a.pbin;
    const u64 total = a.cdf[kCdfBins - 1];
    const u64 cm = bm >= (double)kCdfBins ? total : a.cdf[(int)bm];
    const u64 done_w = tot[C_SEL];
    const double w = (done_w > 0 && cm > 0) ? (double)done_w / (double)cm : a.w0;
    double add = lfac * (double)a.k / w;
    if (add < 1.0) add = 1.0;
    *want_out = cm + (u64)add;
    *m_out = m;
    return 1;
  }
  if (a.mode == PCH_SELECT_DELTA) {
    c->dmode = 1;
    c->use_table = 1;
    c->cutval = from_bits(mn) + delta;
    c->cnt[C_CUT] = bits(c->cutval);
    c->cnt[C_SHIFT] = (u64)(int64_t)-3;
    return 0;
  }
  if (a.mode == PCH_SELECT_STRIDED) {
    // each thread of the partition launch selects the nearest of its windows
    c->smode = 1;
    c->cnt[C_CUT] = (u64)(int64_t)-1;
    c->cnt[C_SHIFT] = (u64)(int64_t)-5;
    return 0;
  }
  const u64 dif = mn ^ mx;
  if (dif == 0) {
    c->shift = 0;
    c->want = mx;
    c->cnt[C_CUT] = mx;
    c->cnt[C_SHIFT] = 0;
    return 0;
  }
  const int hb = 63 - __clzll((long long)dif);
  int s = hb + 1 - 36;
  if (s < 0) s = 0;
  c->shift = (u64)s;
  c->want = (mn >> s) >> 36;  // common prefix above the 36 bits searched
  c->rank = (u64)a.k;
  return 0;
}

// Round set-up, run by one whole wavefront (every lane must call it). For the
// learned cutoff the wavefront finds the smallest CDF bin b with
// cdf[b] >= want in three 64-way steps (65536 = 64 * 64 * 16 bins) and the
// cutoff is the bin's upper edge, above the pool's smallest key.
__device__ void round_begin(const RoundArgs& a, int p) {
  const int lane = lane_id();
  u64 want = 0;
  double m = 0.0;
  int learned = 0;
  if (lane == 0) learned = round_begin_lane0(a, p, &want, &m);
  learned = __shfl(learned, 0, kWave);
  if (!learned) return;
  want = shfl64(want, 0);
  m = shfl_d(m, 0);
  const u64 total = a.cdf[kCdfBins - 1];
  double rho = INFINITY;
  if (want <= total) {
    int lo = (__ffsll((unsigned long long)__ballot((u64)a.cdf[(lane + 1) * 1024 - 1] >= want)) - 1) * 1024;
    lo += (__ffsll((unsigned long long)__ballot((u64)a.cdf[lo + (lane + 1) * 16 - 1] >= want)) - 1) * 16;
    const bool hit = lane < 16 && (u64)a.cdf[lo + (lane < 16 ? lane : 15)] >= want;
    lo += __ffsll((unsigned long long)__ballot(hit)) - 1;
    rho = (double)(lo + 1) * a.pbin;
  }
  if (lane == 0) {
    Ctl* c = a.ctl;
    if (!(rho > m)) rho = m + a.pbin;
    c->lmode = 1;
    c->use_table = 1;
    c->cutval = rho;
    c->cnt[C_CUT] = bits(rho);
    c->cnt[C_SHIFT] = (u64)(int64_t)-4;
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ void k_fill_u64(u64* p, int64_t n, u64 v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_split(Split* p, int64_t n, u64 d, u64 x) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = Split{d, x};
}

__global__ void k_fill_u32(u32* p, int64_t n, u32 v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_set_sources(u64* g, u64* gw, const int32_t* src, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) g[src[i]] = gw[src[i]] = 0ull;
}

// Initialization (Algorithm 1, lines 1-2): every source gets a full fan into
// pool 0 and events for its one-ring into event buffer 0.
__global__ void __launch_bounds__(kBlock) k_init_fans(RoundArgs a, const int32_t* src, int m) {
  u64 kmn = kAllOnes, kmx = 0;
  u32 kept = 0, tiny = 0, ich = 0, defer = 0, notwin = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i - lane_id() < m; i += gridDim.x * kBlock) {
    const bool has = i < m;
    const int v = has ? src[i] : 0;
    const int q0 = has ? a.m.coff[v] : 0;
    const int deg = has ? a.m.coff[v + 1] - q0 : 0;
    wave_fans(a, has, v, q0, deg, 0.0, 0.0, true, 0, 0, kmn, kmx, kept, tiny, ich, defer, notwin);
  }
  kmn = wave_min64(kmn);
  kmx = wave_max64(kmx);
  if (lane_id() == 0) {
    if (kmn != kAllOnes) atomicMin(&a.ctl->kmin[0], kmn);
    if (kmx != 0) atomicMax(&a.ctl->kmax[0], kmx);
  }
}

__global__ void k_begin(RoundArgs a, int p) { round_begin(a, p); }

// Predicted-distance CDFs for the learned cutoff (maximum, histogram, scan)
// of nf fields: field f has n_f predictions at pred + off_f and its table at
// cdf + f (kCdfBins + 1), the bits of the largest positive finite prediction
// in the last word; its bin width goes to pbin[f]. With off == nullptr there
// is one field of n1 predictions at offset 0. blockIdx.y strides over the
// fields. A field's table does not depend on how many fields are built
// together.
struct PredFields {
  const float* pred;
  const int64_t* off;  // [nf] offsets, or null
  const int64_t* n;    // [nf] counts, or null
  int64_t n1;
  int32_t nf;
  u32* cdf;
  double* pbin;  // [nf] or null
};

__device__ __forceinline__ void pred_field(const PredFields& P, int f, const float*& x, int64_t& n, u32*& cdf) {
  x = P.pred + (P.off ? P.off[f] : 0);
  n = P.off ? P.n[f] : P.n1;
  cdf = P.cdf + (int64_t)f * (kCdfBins + 1);
}

__device__ __forceinline__ double pred_bin_width(u32 mx) { return (double)__uint_as_float(mx) * 1.000001 / (double)kCdfBins; }

__global__ void k_pred_max(PredFields P) {
  for (int f = blockIdx.y; f < P.nf; f += gridDim.y) {
    const float* x;
    int64_t n;
    u32* cdf;
    pred_field(P, f, x, n, cdf);
    u32 m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      const float v = x[i];
      const u32 b = (v > 0.f && v < INFINITY) ? __float_as_uint(v) : 0u;  // non-negative floats order as u32
      m = b > m ? b : m;
    }
    atomicMax(&cdf[kCdfBins], m);
  }
}
__global__ void k_pred_hist(PredFields P) {
  for (int f = blockIdx.y; f < P.nf; f += gridDim.y) {
    const float* x;
    int64_t n;
    u32* cdf;
    pred_field(P, f, x, n, cdf);
    const double bw = pred_bin_width(cdf[kCdfBins]);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      const float v = x[i];
      int b = (v > 0.f && bw > 0.0) ? (int)((double)v / bw) : 0;
      if (!(v < INFINITY)) b = kCdfBins - 1;
      b = b < 0 ? 0 : (b >= kCdfBins ? kCdfBins - 1 : b);
      atomicAdd(&cdf[b], 1u);
    }
  }
}
__global__ void __launch_bounds__(1024) k_pred_scan(PredFields P) {
  __shared__ u32 part[1024];
  constexpr int per = kCdfBins / 1024;
  for (int f = blockIdx.x; f < P.nf; f += gridDim.x) {
    u32* hist = P.cdf + (int64_t)f * (kCdfBins + 1);
    u32 loc[per];
    u32 sum = 0;
    for (int i = 0; i < per; ++i) {
      loc[i] = hist[threadIdx.x * per + i];
      sum += loc[i];
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const u32 y = threadIdx.x >= (u32)o ? part[threadIdx.x - o] : 0u;
      __syncthreads();
      part[threadIdx.x] += y;
      __syncthreads();
    }
    u32 run = part[threadIdx.x] - sum;
    for (int i = 0; i < per; ++i) {
      run += loc[i];
      hist[threadIdx.x * per + i] = run;
    }
    if (threadIdx.x == 0 && P.pbin) P.pbin[f] = pred_bin_width(hist[kCdfBins]);
    __syncthreads();
  }
}

// Enqueues the tables of P (zeroed first).
void enqueue_pred_cdf(const PredFields& P, hipStream_t st) {
  k_fill_u32<<<256, kBlock, 0, st>>>(P.cdf, (int64_t)P.nf * (kCdfBins + 1), 0u);
  const unsigned fy = (unsigned)std::min(P.nf, 65535);
  k_pred_max<<<dim3(P.off ? 16 : 256, fy), kBlock, 0, st>>>(P);
  k_pred_hist<<<dim3(P.off ? 64 : 1024, fy), kBlock, 0, st>>>(P);
  k_pred_scan<<<std::min(P.nf, 65535), 1024, 0, st>>>(P);
}

// One 12-bit radix-select pass over the truncated keys t = key_bits >> shift:
// pass 0 bins bits 35..24, pass 1 bits 23..12, pass 2 bits 11..0, counting
// only keys whose higher bits equal the prefix chosen so far. The last block
// to finish finds the bin holding the remaining rank, extends the prefix and
// clears the histogram.
__global__ void __launch_bounds__(kBlock) k_hist(RoundArgs a, int p, int pass) {
  __shared__ u32 h[kHistBins];
  __shared__ u32 part[kBlock];
  __shared__ u32 pick_bin, pick_before;
  __shared__ int is_last;
  Ctl* c = a.ctl;
  if (!c->active || c->use_table || c->sel_all || c->rank == 0) return;
  for (int i = threadIdx.x; i < kHistBins; i += kBlock) h[i] = 0;
  __syncthreads();
  const u64 N = min(c->nscan, (u64)a.cap);
  const int s = (int)c->shift;
  const int lo = 24 - 12 * pass;
  const u64 want = c->want;
  // tombstones (key kDead) never match a prefix of a finite key
  const double2* sk = c->pin ? a.pool[1].sk : a.pool[0].sk;
  for (u64 i = blockIdx.x * (u64)kBlock + threadIdx.x; i < N; i += (u64)gridDim.x * kBlock) {
    const u64 t = bits(sk[i].y) >> s;
    if ((t >> (lo + 12)) == want) atomicAdd(&h[(t >> lo) & (kHistBins - 1)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHistBins; i += kBlock)
    if (h[i]) atomicAdd(&a.hist[i], h[i]);
  // The last workgroup reads the histogram with device-scope atomic loads:
  // waiting for this wavefront's atomics orders them before the ticket (as in
  // k_events3; no cache write-back is needed).
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(&c->ticket, 1ull) == (u64)(gridDim.x - 1);
  __syncthreads();
  if (!is_last) return;
  constexpr int per = kHistBins / kBlock;
  u32 loc[per];
  u32 sum = 0;
  for (int i = 0; i < per; ++i) {
    loc[i] = __hip_atomic_load(&a.hist[threadIdx.x * per + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sum += loc[i];
  }
  if (threadIdx.x == 0) {
    pick_bin = 0;
    pick_before = 0;
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    const u32 y = threadIdx.x >= (u32)o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  const u64 rank = c->rank;
  const u32 incl = part[threadIdx.x];
  const u32 excl = incl - sum;
  if (excl < rank && rank <= incl) {
    u32 run = excl;
    for (int i = 0; i < per; ++i) {
      if (run + loc[i] >= rank) {
        pick_bin = threadIdx.x * per + i;
        pick_before = run;
        break;
      }
      run += loc[i];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHistBins; i += kBlock) a.hist[i] = 0;
  if (threadIdx.x == 0) {
    c->want = (want << 12) | pick_bin;
    c->rank = rank - pick_before;
    c->ticket = 0;
    if (pass == 2) c->cnt[C_CUT] = c->want, c->cnt[C_SHIFT] = c->shift;
  }
}

// Split the pool (selection, Section 4.2 step 1): stale windows (sigma >
// geod_dist of their pseudo-source) are dropped, selected windows go to the
// selection buffer, the rest stay in the pool. In a round that keeps the pool
// in place, a kept window is not moved: only the selected and stale ones are
// touched (copied out and marked as tombstones), so the scan reads the key,
// distance and pseudo-source of each slot and nothing else. A compacting round
// moves the kept windows into the other buffer instead. Appends are reserved
// per wavefront.
__device__ __forceinline__ void ph_partition(const RoundArgs& a, int p, u64 t0, u64 stride) {
  Ctl* c = a.ctl;
  const bool active = c->active != 0;
  const u64 pin = c->pin, pout = c->pout;
  const u64 N = active ? min(c->nscan, (u64)a.cap) : 0;
  const int s = (int)c->shift;
  const u64 T = c->want;
  const bool all = c->sel_all;
  const bool tab = c->use_table;
  const double cv = c->cutval;
  const bool strided = c->smode != 0;
  const bool inplace = pin == pout;
  const Pool P = pin ? a.pool[1] : a.pool[0];
  const Pool Q = pout ? a.pool[1] : a.pool[0];
  u64* qctr = &c->npool[pout & 1];
  const Pool S = a.sel;
  // Strided selection (Section 6, the approximate k-selection): the thread
  // owns slots t0, t0 + stride, t0 + 2 stride, ... and selects the nearest
  // of its live windows that are not stale (the first one on equal keys).
  u64 imin = kAllOnes;
  if (strided) {
    double kbest = 0.0;
    for (u64 i = t0; i < N; i += stride) {
      const double2 wsk = P.sk[i];
      if (bits(wsk.y) == kDead) continue;
      const int32_t src = P.es[i].y;
      if (!idx_ok(c, src, a.m.nv)) continue;
      if (wsk.x > from_bits(lda(&a.s.g[src]))) continue;  // stale
      if (imin == kAllOnes || wsk.y < kbest) {
        kbest = wsk.y;
        imin = i;
      }
    }
  }
  u32 stale_n = 0, kept_in = 0;
  u64 kmn = kAllOnes, kmx = 0;
  for (u64 i = t0; i - lane_id() < N; i += stride) {
    bool sel = false, keep = false, gone = false;
    double2 wsk = make_double2(0.0, 0.0);
    int2 wes = make_int2(0, 0);
    if (i < N) {
      wsk = P.sk[i];
      if (bits(wsk.y) != kDead) {
        wes = P.es[i];
        const bool stale = !idx_ok(c, wes.y, a.m.nv) || wsk.x > from_bits(lda(&a.s.g[wes.y]));
        if (stale) {
          stale_n++;
          gone = true;
        } else {
          sel = strided ? (all || i == imin) : (tab ? (wsk.y <= cv) : (all || ((bits(wsk.y) >> s) <= T)));
          keep = !sel;
        }
      }
    }
    const bool move = sel || (keep && !inplace);
    double2 wbb = make_double2(0.0, 0.0), wpp = wbb;
    if (move) {
      wbb = P.bb[i];
      wpp = P.pp[i];
    }
    u64 js, jk, jz;
    u32 ts, tk, tz;
    wave_reserve3(&c->nsel, sel ? 1u : 0u, qctr, (keep && !inplace) ? 1u : 0u, &c->nsel, 0u, js, jk, jz, ts, tk,
                  tz);
    if (sel) {
      if (js < (u64)a.cap) {
        store_window(S, js, wbb.x, wbb.y, wpp.x, wpp.y, wsk.x, wsk.y, wes.x, wes.y);
        if (a.org_shift >= 0) atomicAdd(&a.org_hist[wes.x >> a.org_shift], 1u);
      } else {
        flag_overflow(c);
      }
    }
    if (inplace && (sel || gone)) reinterpret_cast<double*>(P.sk)[2 * i + 1] = from_bits(kDead);
    if (keep) {
      if (inplace) {
        kept_in++;
      } else if (jk < (u64)a.cap) {
        store_window(Q, jk, wbb.x, wbb.y, wpp.x, wpp.y, wsk.x, wsk.y, wes.x, wes.y);
      } else {
        flag_overflow(c);
      }
      const u64 kb = bits(wsk.y);
      kmn = kb < kmn ? kb : kmn;
      kmx = kb > kmx ? kb : kmx;
    }
  }
  u32 tot[2] = {stale_n, kept_in};
  block_totals(kmn, kmx, tot);
  if (threadIdx.x == 0) {
    if (kmn != kAllOnes) atomicMin(&c->kmin[1 - p], kmn);
    if (kmx != 0) atomicMax(&c->kmax[1 - p], kmx);
    if (tot[0] && a.counts) atomicAdd(&c->cnt[C_STALE], (u64)tot[0]);
    if (tot[1]) atomicAdd(&c->keptin, (u64)tot[1]);
  }
}

__global__ void __launch_bounds__(kBlock) k_partition(RoundArgs a, int p) {
  ph_partition(a, p, blockIdx.x * (u64)kBlock + threadIdx.x, (u64)gridDim.x * kBlock);
}

// Per-launch values of the propagation that every window reads.
struct PropCtx {
  Pool Q;    // the next round's pool
  u64* qctr; // its slot counter
  DistEv E;  // this round's distance events
  int sh;    // selection test of a child: key bits >> sh <= T, or key <= cv
  u64 T;
  bool all, tab;
  double cv;
};

// A window a lane keeps in registers for its next propagation step (the
// first child of its last window that hops on).
struct RegWin {
  bool has = false;
  double2 bb, pp;
  double sg;
  int2 es;
};

// A lane's counts over the windows it propagated.
struct PropAcc {
  u32 n_tiny = 0, n_ich = 0, n_notwin = 0, n_nonfin = 0, n_kids = 0, n_dev = 0, n_aev = 0;
  u64 kmn = kAllOnes, kmx = 0;
};

// Algorithm 2 for one lane's window (have = false: the lane has none, but
// still takes part in the reservations, so every lane of the wavefront, or
// of the workgroup with kBlockRes, calls this). Children that pass the
// round's selection test go to HQ (capacity hq_cap) through the counter
// nq_ctr when to_hop is set, the others to the next pool; events go to this
// round's buffers.
template <bool kBlockRes, class HopQ, bool kReg = false, int BS = kBlock>
__device__ __forceinline__ void prop_window(const RoundArgs& a, int p, const PropCtx& x, bool have, double2 wbb,
                                            double2 wpp, double2 wsk, int2 wes, bool to_hop, const HopQ& HQ,
                                            u64* nq_ctr, u64 hq_cap, PropAcc& acc, RegWin* rw = nullptr) {
  Ctl* c = a.ctl;
  const DevMesh& m = a.m;
  const u64* g = a.s.g;
  // outputs of this lane, in fixed slots (no per-lane arrays, which would
  // live in scratch memory): the left and right child, and the distance
  // events at v0, v1 and v2
  bool cl = false, cr = false;
  double lb0 = 0, lb1 = 0, lpx = 0, lpy = 0, lkey = 0, rb0 = 0, rb1 = 0, rpx = 0, rpy = 0, rkey = 0;
  int32_t le = 0, re = 0;
  bool e0 = false, e1 = false, e2 = false;
  int32_t ev0 = 0, ev1 = 0, ev2 = 0;
  double ed0 = 0, ed1 = 0, ed2 = 0, epx = 0, epy = 0;
  int32_t eq0 = -1, eq1 = -1, eq2 = -1;  // angle recipes (see DistEv)
  bool has_aev = false;
  double aD = 0, aX = 0;
  double sg = 0;
  int32_t src = 0, e = 0;
  if (have && idx_ok(c, wes.x, m.nh) && idx_ok(c, wes.y, m.nv)) {
    const double b0 = wbb.x, b1 = wbb.y, px = wpp.x, py = wpp.y;
    epx = px;
    epy = py;
    sg = wsk.x;
    e = wes.x;
    src = wes.y;
    // everything that depends on e only, in one batch of loads
    const pch::HalfEdge h = m.hl[e].h;
    const pch::HalfEdgeAng ha = m.hl[e].a;
    const u64 ad_bits = lda(&a.s.as[e].D);
    const u64 ax_bits = lda(&a.s.as[e].X);
    const double L = h.L, x2 = h.x2, y2 = h.y2, l02 = h.l02, l12 = h.l12;
    const int v0 = h.v0, v1 = h.v1, v2 = h.v2;
    const double g0 = from_bits(lda(&g[v0])), g1 = from_bits(lda(&g[v1])), g2 = from_bits(lda(&g[v2]));
    const double tol = kTau * L;
    // stronger filtering (filters bit 3): the window takes the two endpoint
    // tests of the ICH filter again, against the round-start distances, which
    // may have dropped since it was made; both hold for any window on an edge
    // (along the edge, |I x| - |v0 x| never increases toward v1 and
    // |I x| - |v1 x| never increases toward v0), so a window that fails one is
    // beaten on its whole interval
    bool drop = false;
    if (a.retest) {
      const double dx1 = b1 - px;
      const double f1 = sg + sqrt(dx1 * dx1 + py * py);
      const double dx0 = b0 - px;
      const double f0 = sg + sqrt(dx0 * dx0 + py * py);
      drop = f1 > (g0 + b1) * kFm || f0 > (g1 + (L - b0)) * kFm;
    }
    if (drop) acc.n_ich++;
    if (!drop) {
      const double den = y2 - py;
      const double t = (-py) / den;
      const double X = px + (x2 - px) * t;
      if (!isfinite(X)) acc.n_nonfin++;
      const bool occ = (X >= b0 - tol) && (X <= b1 + tol);
      // Every candidate value is computed before the decisions that use it,
      // with no branch between the divisions and square roots, so that the
      // independent chains of the three events and of both children overlap
      // (a wavefront's lanes take different branches anyway). Each value is
      // the same expression as where it is used; unused ones are dropped.
      const double dE0 = sg + sqrt(px * px + py * py);
      const double ex1 = px - L;
      const double dE1 = sg + sqrt(ex1 * ex1 + py * py);
      const double ax = x2 - px, ay = y2 - py;
      const double d2 = sg + sqrt(ax * ax + ay * ay);
      // left child, on the edge from v0 to v2
      const double qL0 = (py * b0) / (x2 * py + y2 * (b0 - px));
      const double qL1 = (py * b1) / (x2 * py + y2 * (b1 - px));
      double cL0 = (b0 == 0.0 ? 0.0 : qL0) * l02, cL1 = (occ ? 1.0 : qL1) * l02;
      if (cL0 < 0.0) cL0 = 0.0;
      if (cL1 > l02) cL1 = l02;
      const double uLx = ha.ulx, uLy = ha.uly;  // x2 / l02, y2 / l02
      const double pLx = uLx * px + uLy * py;
      double pLy = uLx * py - uLy * px;
      if (pLy > 0.0) pLy = 0.0;
      const double rLx = uLx * cL0 - L, rLy = uLy * cL0;
      const double rLd = sqrt(rLx * rLx + rLy * rLy);
      const int fL = child_filter(cL0, cL1, pLx, pLy, sg, l02, g0, g2, true, true, g1, rLd, a.eps, a.ich_on);
      const double kL = window_key(cL0, cL1, pLx, pLy, sg);
      // right child, on the edge from v2 to v1
      const double ex = L - x2;
      const double qR0 = ((x2 * py - py * b0) + y2 * (b0 - px)) / (y2 * (b0 - px) - ex * py);
      const double qR1 = ((x2 * py - py * b1) + y2 * (b1 - px)) / (y2 * (b1 - px) - ex * py);
      double cR0 = (occ ? 0.0 : qR0) * l12, cR1 = (b1 == L ? 1.0 : qR1) * l12;
      if (cR0 < 0.0) cR0 = 0.0;
      if (cR1 > l12) cR1 = l12;
      const double uRx = ha.urx, uRy = ha.ury;  // (L - x2) / l12, (-y2) / l12
      const double qx = px - x2, qy = py - y2;
      const double pRx = uRx * qx + uRy * qy;
      double pRy = uRx * qy - uRy * qx;
      if (pRy > 0.0) pRy = 0.0;
      const double rRx = x2 + uRx * cR1, rRy = y2 + uRy * cR1;
      const double rRd = sqrt(rRx * rRx + rRy * rRy);
      const int fR = child_filter(cR0, cR1, pRx, pRy, sg, l12, g2, g1, true, false, g0, rRd, a.eps, a.ich_on);
      const double kR = window_key(cR0, cR1, pRx, pRy, sg);
      // the decisions
      if (b0 <= tol && dE0 < g0 * kEv) {
        e0 = true;
        ev0 = v0;
        ed0 = dE0;
        eq0 = (h.pflags & 1) ? (e << 2) : -1;
      }
      if (b1 >= L - tol && dE1 < g1 * kEv) {
        e1 = true;
        ev1 = v1;
        ed1 = dE1;
        eq1 = (h.pflags & 2) ? ((e << 2) | 1) : -1;
      }
      bool doL = false, doR = false;
      if (occ) {
        if (d2 < g2 * kEv) {
          e2 = true;
          ev2 = v2;
          ed2 = d2;
          eq2 = (h.pflags & 4) ? ((e << 2) | 2) : -1;
        }
        if (!a.ch_on) {
          doL = doR = true;
        } else {
          const double Ds = from_bits(ad_bits);
          const double Xs = from_ordkey(ax_bits);
          if (d2 < Ds) {
            has_aev = true;
            aD = d2;
            aX = X;
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
        if (h.tl < 0) {
          acc.n_notwin++;
        } else if (fL == 1) {
          acc.n_tiny++;
        } else if (fL == 2) {
          acc.n_ich++;
        } else {
          cl = true;
          lb0 = cL0;
          lb1 = cL1;
          lpx = pLx;
          lpy = pLy;
          lkey = kL;
          le = h.tl;
        }
      }
      if (doR) {
        if (h.tr < 0) {
          acc.n_notwin++;
        } else if (fR == 1) {
          acc.n_tiny++;
        } else if (fR == 2) {
          acc.n_ich++;
        } else {
          cr = true;
          rb0 = cR0;
          rb1 = cR1;
          rpx = pRx;
          rpy = pRy;
          rkey = kR;
          re = h.tr;
        }
      }
    }
  }
  // children that pass the round's selection test go to the next hop
  const bool ql = cl && to_hop && (x.tab ? (lkey <= x.cv) : (x.all || ((bits(lkey) >> x.sh) <= x.T)));
  const bool qr = cr && to_hop && (x.tab ? (rkey <= x.cv) : (x.all || ((bits(rkey) >> x.sh) <= x.T)));
  const int nk = (cl ? 1 : 0) + (cr ? 1 : 0);
  const int nh = (ql ? 1 : 0) + (qr ? 1 : 0);  // children that hop on
  // with kReg the first of them stays in the lane's registers (rw), the
  // second goes to the hop list
  const int nq = kReg ? (nh > 1 ? 1 : 0) : nh;
  const int nd = (e0 ? 1 : 0) + (e1 ? 1 : 0) + (e2 ? 1 : 0);
  // append children, distance events and angle events (one reservation per
  // wavefront each)
  u32 tk, td, ta, tq;
  u64 jk, jd, ja, jq;
  if constexpr (kBlockRes)
    block_reserve4<BS>(x.qctr, (u32)(nk - nh), &c->ndev[p], (u32)nd, &c->naev, has_aev ? 1u : 0u, nq_ctr,
                   (u32)nq, jk, jd, ja, jq, tk, td, ta, tq);
  else
    wave_reserve4(x.qctr, (u32)(nk - nh), &c->ndev[p], (u32)nd, &c->naev, has_aev ? 1u : 0u, nq_ctr,
                  (u32)nq, jk, jd, ja, jq, tk, td, ta, tq);
  if constexpr (kReg) rw->has = false;
  auto put_child = [&](bool toq, double cb0, double cb1, double cpx, double cpy, double ckey, int32_t ce) {
    if constexpr (kReg) {
      if (toq && !rw->has) {
        rw->has = true;
        rw->bb = make_double2(cb0, cb1);
        rw->pp = make_double2(cpx, cpy);
        rw->sg = sg;
        rw->es = make_int2(ce, src);
        return;
      }
    }
    if (toq) {
      const u64 j = jq++;
      if (j < hq_cap)
        store_window(HQ, j, cb0, cb1, cpx, cpy, sg, ckey, ce, src);
      else
        flag_overflow(c);
      return;
    }
    const u64 j = jk++;
    if (j < (u64)a.cap) {
      store_window(x.Q, j, cb0, cb1, cpx, cpy, sg, ckey, ce, src);
      const u64 kb = bits(ckey);
      acc.kmn = kb < acc.kmn ? kb : acc.kmn;
      acc.kmx = kb > acc.kmx ? kb : acc.kmx;
    } else {
      flag_overflow(c);
    }
  };
  if (cl) put_child(ql, lb0, lb1, lpx, lpy, lkey, le);
  if (cr) put_child(qr, rb0, rb1, rpx, rpy, rkey, re);
  // the incoming angle of an event at a pseudo-source is evaluated later,
  // only for the events that win their vertex (event_angle)
  // each event lowers geod_dist's write copy at once and is recorded for
  // the event passes (winners, fans)
  auto put_event = [&](int32_t v, double dv, int32_t q) {
    atomicMin(&a.s.gw[v], bits(dv));
    const u64 j = jd++;
    if (j < (u64)a.ecap) {
      x.E.vq[j] = make_int2(v, q);
      x.E.d[j] = dv;
      x.E.xy[j] = q >= 0 ? make_double2(epx, epy) : make_double2(0.0, 0.0);
    } else {
      flag_overflow(c);
    }
  };
  if (e0) put_event(ev0, ed0, eq0);
  if (e1) put_event(ev1, ed1, eq1);
  if (e2) put_event(ev2, ed2, eq2);
  if (has_aev) {
    // the corner's write copy takes the apex distance at once; a corner whose
    // distance improves forgets its old crossing (the crossings are compared
    // in the second event pass)
    if (atomicMin(&a.s.asw[e].D, bits(aD)) > bits(aD)) a.s.asw[e].X = kAllOnes;
    if (ja < (u64)a.acap) {
      a.aev.e[ja] = e;
      a.aev.D[ja] = aD;
      a.aev.X[ja] = aX;
    } else {
      flag_overflow(c);
    }
  }
  // wavefront totals (the same on every lane), counted once by lane 0
  if (lane_id() == 0) {
    acc.n_kids += tk + tq;
    acc.n_dev += td;
    acc.n_aev += ta;
  }
  if constexpr (kReg) acc.n_kids += rw->has ? 1u : 0u;  // each lane its register child
}

// End of a propagation launch: the workgroup's key range and counts.
__device__ __forceinline__ void prop_finish(const RoundArgs& a, int p, PropAcc& acc) {
  Ctl* c = a.ctl;
  u64 kmn = acc.kmn, kmx = acc.kmx;
  u32 tot[7] = {acc.n_tiny, acc.n_ich, acc.n_notwin, acc.n_nonfin, acc.n_kids, acc.n_dev, acc.n_aev};
  block_totals(kmn, kmx, tot);
  if (threadIdx.x == 0) {
    if (kmn != kAllOnes) atomicMin(&c->kmin[1 - p], kmn);
    if (kmx != 0) atomicMax(&c->kmax[1 - p], kmx);
    if (tot[3]) atomicAdd(&c->nonfinite, (u64)tot[3]);
    if (a.counts) {
      if (tot[0]) atomicAdd(&c->cnt[C_TINY], (u64)tot[0]);
      if (tot[1]) atomicAdd(&c->cnt[C_ICH], (u64)tot[1]);
      if (tot[2]) atomicAdd(&c->xcnt[X_NOTWIN], (u64)tot[2]);
      if (tot[4]) atomicAdd(&c->cnt[C_KIDS], (u64)tot[4]);
      if (tot[5]) atomicAdd(&c->cnt[C_DEV], (u64)tot[5]);
      if (tot[6]) atomicAdd(&c->cnt[C_AEV], (u64)tot[6]);
    }
  }
}

// Algorithm 2 for every selected window, against the round-start geod_dist
// and angle_split (delayed update, Remark 3). Hop 1 takes the windows the
// partition selected. With hops > 1 a child that passes the round's own
// selection test is queued for the next hop of the same round instead of
// entering the pool, and hop h >= 2 propagates hop h - 1's queue, still
// against the round-start values: the order in which windows propagate does
// not change the distances, and stale values only prune less.
__device__ __forceinline__ void ph_propagate(const RoundArgs& a, int p, int hop, u64 t0, u64 stride) {
  Ctl* c = a.ctl;
  const Pool S = hop > 1 ? a.hq[hop & 1] : (a.org_shift >= 0 ? a.sorted : a.sel);
  // The lane's first window is loaded together with the round's counters (an
  // index below cap is always in bounds), so the two round trips overlap.
  double2 f_bb = make_double2(0, 0), f_pp = f_bb, f_sk = f_bb;
  int2 f_es = make_int2(0, 0);
  if (t0 < (u64)a.cap) {
    f_bb = S.bb[t0];
    f_pp = S.pp[t0];
    f_sk = S.sk[t0];
    f_es = S.es[t0];
  }
  const bool active = c->active != 0;
  const u64 n_in = hop <= 1 ? c->nsel : c->nhop[hop - 1];
  const u64 N = active ? min(n_in, (u64)a.cap) : 0;
  const u64 pout = c->pout;
  const Pool Q = pout ? a.pool[1] : a.pool[0];
  // children hop on when they pass the round's selection test; a strided
  // round has no key test, so its children wait for the next round
  const bool to_hop = hop < a.hops && c->smode == 0;
  const Pool HQ = a.hq[(hop + 1) & 1];
  u64* nq_ctr = &c->nhop[hop < kMaxHops ? hop : kMaxHops];
  const int sh = (int)c->shift;
  const u64 T = c->want;
  const bool all = c->sel_all;
  const bool tab = c->use_table;
  const double cv = c->cutval;
  const PropCtx x{Q, &c->npool[pout & 1], a.ev[p], sh, T, all, tab, cv};
  if (t0 == 0 && active) {
    if (hop <= 1) {
      c->cnt[C_SEL] = n_in;
      if (a.counts) atomicAdd(&c->xcnt[X_SEL1], n_in);
    } else {
      c->cnt[C_SEL] = c->cnt[C_SEL] + n_in;
    }
  }
  PropAcc acc;
  for (u64 i = t0; i - lane_id() < N; i += stride) {
    const bool have = i < N;
    double2 wbb = f_bb, wpp = f_pp, wsk = f_sk;
    int2 wes = f_es;
    if (have && i != t0) {
      wbb = S.bb[i];
      wpp = S.pp[i];
      wsk = S.sk[i];
      wes = S.es[i];
    }
    prop_window<false, Pool>(a, p, x, have, wbb, wpp, wsk, wes, to_hop, HQ, nq_ctr, (u64)a.cap, acc);
  }
  prop_finish(a, p, acc);
}

// Organization by edge (Algorithm 3's reorganization, here as a one-pass
// bucket sort): exclusive scan of the per-bucket counts of the selected
// windows into slot offsets, clearing the counts for the next round.
__global__ void __launch_bounds__(1024) k_org_scan(RoundArgs a) {
  __shared__ u32 part[1024];
  if (!a.ctl->active) return;
  constexpr int per = kOrgBuckets / 1024;
  u32 loc[per];
  u32 sum = 0;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    loc[i] = a.org_hist[threadIdx.x * per + i];
    a.org_hist[threadIdx.x * per + i] = 0u;
    sum += loc[i];
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const u32 y = threadIdx.x >= (u32)o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  u32 run = part[threadIdx.x] - sum;
#pragma unroll
  for (int i = 0; i < per; ++i) {
    a.org_ofs[threadIdx.x * per + i] = run;
    run += loc[i];
  }
}

// Scatter of the selected windows into their bucket's slots: windows on
// nearby half-edges (nearby faces) end up next to each other, so neighbouring
// lanes of the propagation read neighbouring half-edge records and vertices.
__global__ void __launch_bounds__(kBlock) k_org_scatter(RoundArgs a) {
  Ctl* c = a.ctl;
  if (!c->active) return;
  const u64 N = min(c->nsel, (u64)a.cap);
  const Pool S = a.sel, D = a.sorted;
  for (u64 i = blockIdx.x * (u64)kBlock + threadIdx.x; i < N; i += (u64)gridDim.x * kBlock) {
    const int2 es = S.es[i];
    const u64 j = atomicAdd(&a.org_ofs[es.x >> a.org_shift], 1u);
    D.bb[j] = S.bb[i];
    D.pp[j] = S.pp[i];
    D.sk[j] = S.sk[i];
    D.es[j] = es;
  }
}

__global__ void __launch_bounds__(kBlock) k_propagate(RoundArgs a, int p, int hop) {
  ph_propagate(a, p, hop, blockIdx.x * (u64)kBlock + threadIdx.x, (u64)gridDim.x * kBlock);
}

constexpr int kFuseHops = 6;          // hops that one fused launch carries
constexpr int kFuseCap = 2 * kBlock;  // windows a hop list in LDS holds

// The pool scan of the fused launches deals the pool in 64-slot chunks,
// round-robin over the G workgroups, newest chunks first: ticket t stands for
// workgroup slot t % G of deal t / G, in which wave w of the workgroup scans
// chunk M - 1 - (((t / G) nW + w) G + t % G) of the pool's M chunks. The
// newest windows, which hold most of a round's selected ones, sit together
// at the end of the pool; dealt this way they spread over every workgroup
// instead of loading a few with long hop chains, and they are dealt first,
// so the chunks with the longest hop chains start first and the light ones
// fill in at the end. Each workgroup takes ticket blockIdx.x first and then
// the next free one from a counter, so workgroups whose windows hop little
// scan more. Called by the whole workgroup (uniformly); returns false once
// the workgroup's ticket lies past the pool, else sets i to this thread's
// slot (N for a wave whose chunk lies past the pool).
__device__ __forceinline__ bool scan_ticket(Ctl* c, u64 N, u32 G, u32 nW, bool& first, u32& ticket, u32* s_ticket,
                                            u64& i) {
  if (!first) {
    if (threadIdx.x == 0) *s_ticket = (u32)atomicAdd(&c->scan_next, 1ull) + G;
    __syncthreads();
    ticket = *s_ticket;
  }
  first = false;
  const u64 deal = ticket / G, slot = ticket % G;
  const u64 M = (N + kWave - 1) / kWave;
  if (deal * nW * G + slot >= M) return false;
  const u64 kc = (deal * nW + threadIdx.x / kWave) * G + slot;
  i = kc < M ? (M - 1 - kc) * kWave + lane_id() : N;
  return true;
}



// All hops of a round in one launch (hops <= NL + 1 <= kFuseHops). Each
// workgroup propagates its share of the selected windows and, depth first,
// the children that pass the round's selection test, from NL per-hop lists in
// LDS: every step takes up to kBlock windows from the deepest non-empty list
// (its next chunk of the selection when all lists are empty) and appends
// their hopping children to the next hop's list. A list is filled only while
// every deeper list is empty, from at most kBlock windows, so it never holds
// more than 2 * kBlock. Every window propagates at the hop it would reach
// with one launch per hop, against the same round-start values, so the
// round's windows, events and counts are the same; hops - 1 launches and
// their ramps are saved per round. The lists take NL * 24 KiB of LDS, so
// fewer hops leave room for more workgroups per compute unit.
template <int NL>
__global__ void __launch_bounds__(kBlock) k_propagate_fused(RoundArgs a, int p) {
  __shared__ double2 l_bb[NL][kFuseCap], l_pp[NL][kFuseCap];
  __shared__ double l_sg[NL][kFuseCap];
  __shared__ int2 l_es[NL][kFuseCap];
  __shared__ u64 l_n[NL + 2];  // l_n[h]: windows in the list of hop h (h >= 2)
  constexpr int kTop = NL + 1;  // the deepest hop
  Ctl* c = a.ctl;
  const u64 t0 = blockIdx.x * (u64)kBlock + threadIdx.x, stride = (u64)gridDim.x * kBlock;
  const Pool S = a.org_shift >= 0 ? a.sorted : a.sel;
  // the lane's first window is loaded together with the round's counters
  double2 f_bb = make_double2(0, 0), f_pp = f_bb, f_sk = f_bb;
  int2 f_es = make_int2(0, 0);
  if (t0 < (u64)a.cap) {
    f_bb = S.bb[t0];
    f_pp = S.pp[t0];
    f_sk = S.sk[t0];
    f_es = S.es[t0];
  }
  if (threadIdx.x <= (unsigned)kTop) l_n[threadIdx.x] = 0;
  const bool active = c->active != 0;
  const u64 n_in = c->nsel;
  const u64 N = active ? min(n_in, (u64)a.cap) : 0;
  // a strided round has no key test, so its children wait for the next round
  const bool hop_ok = c->smode == 0;
  const int sh = (int)c->shift;
  const u64 T = c->want;
  const bool all = c->sel_all;
  const bool tab = c->use_table;
  const double cv = c->cutval;
  const u64 pout = c->pout;
  const PropCtx x{pout ? a.pool[1] : a.pool[0], &c->npool[pout & 1], a.ev[p], sh, T, all, tab, cv};
  const int hops = a.hops < kTop ? a.hops : kTop;
  if (t0 == 0 && active) {
    atomicAdd(&c->cnt[C_SEL], n_in);
    if (a.counts) atomicAdd(&c->xcnt[X_SEL1], n_in);
  }
  __syncthreads();
  PropAcc acc;
  u64 base = blockIdx.x * (u64)kBlock;  // the workgroup's next chunk of the selection
  u64 hopped = 0;                       // windows taken from the lists (thread 0)
  int lvl = 1;                          // hop of the next step (the same in every thread)
  for (;;) {
    bool have;
    double2 wbb = f_bb, wpp = f_pp, wsk = f_sk;
    int2 wes = f_es;
    if (lvl == 1) {
      if (base >= N) break;
      const u64 i = base + threadIdx.x;
      have = i < N;
      if (have && i != t0) {
        wbb = S.bb[i];
        wpp = S.pp[i];
        wsk = S.sk[i];
        wes = S.es[i];
      }
      base += stride;
    } else {
      const u64 n = l_n[lvl];
      const u64 take = n < (u64)kBlock ? n : (u64)kBlock;
      have = threadIdx.x < take;
      if (have) {
        const u64 j = n - take + threadIdx.x;
        wbb = l_bb[lvl - 2][j];
        wpp = l_pp[lvl - 2][j];
        wsk = make_double2(l_sg[lvl - 2][j], 0.0);
        wes = l_es[lvl - 2][j];
      }
      __syncthreads();  // every thread has its window before the list shrinks
      if (threadIdx.x == 0) {
        l_n[lvl] = n - take;
        hopped += take;
      }
    }
    const int nl = lvl < kTop ? lvl + 1 : kTop;
    const HopList HQ{l_bb[nl - 2], l_pp[nl - 2], l_sg[nl - 2], l_es[nl - 2]};
    prop_window<true, HopList>(a, p, x, have, wbb, wpp, wsk, wes, hop_ok && lvl < hops, HQ, &l_n[nl],
                               (u64)kFuseCap, acc);
    __syncthreads();  // the next list and its length are visible
    if (lvl < hops && l_n[lvl + 1] != 0) {
      ++lvl;
    } else {
      while (lvl > 1 && l_n[lvl] == 0) --lvl;
    }
  }
  if (threadIdx.x == 0 && hopped != 0) atomicAdd(&c->cnt[C_SEL], hopped);
  prop_finish(a, p, acc);
}

// Selection and propagation in one launch (hops <= NL + 1): the workgroups
// scan the pool as the partition does (stale windows dropped, the kept ones
// left in place or compacted into the other buffer) and propagate each
// selected window in the same step, without a selection buffer; the hopping
// children then go depth first through the LDS lists as in
// k_propagate_fused. The selected windows, their order aside, and every
// count are those of the partition followed by the propagation, against the
// same round-start values.
template <int NL>
__global__ void __launch_bounds__(kBlock) k_select_propagate(RoundArgs a, int p) {
  __shared__ double2 l_bb[NL][kFuseCap], l_pp[NL][kFuseCap];
  __shared__ double l_sg[NL][kFuseCap];
  __shared__ int2 l_es[NL][kFuseCap];
  __shared__ u64 l_n[NL + 2];  // l_n[h]: windows in the list of hop h (h >= 2)
  constexpr int kTop = NL + 1;  // the deepest hop
  Ctl* c = a.ctl;
  if (threadIdx.x <= (unsigned)kTop) l_n[threadIdx.x] = 0;
  const bool active = c->active != 0;
  const u64 pin = c->pin, pout = c->pout;
  const u64 N = active ? min(c->nscan, (u64)a.cap) : 0;
  const int sh = (int)c->shift;
  const u64 T = c->want;
  const bool all = c->sel_all;
  const bool tab = c->use_table;
  const double cv = c->cutval;
  const bool inplace = pin == pout;
  const Pool P = pin ? a.pool[1] : a.pool[0];
  const PropCtx x{pout ? a.pool[1] : a.pool[0], &c->npool[pout & 1], a.ev[p], sh, T, all, tab, cv};
  const int hops = a.hops < kTop ? a.hops : kTop;
  __syncthreads();
  PropAcc acc;
  u32 stale_n = 0, kept_in = 0, n_sel = 0;
  __shared__ u32 s_ticket;
  bool first = true;
  u32 ticket = blockIdx.x;  // the workgroup's deal of the pool (scan_ticket)
  u64 hopped = 0;           // windows taken from the lists (thread 0)
  int lvl = 1;              // hop of the next step (the same in every thread)
  for (;;) {
    bool have = false;
    double2 wbb = make_double2(0.0, 0.0), wpp = wbb, wsk = wbb;
    int2 wes = make_int2(0, 0);
    if (lvl == 1) {
      u64 i = 0;
      if (!scan_ticket(c, N, gridDim.x, kBlock / kWave, first, ticket, &s_ticket, i)) break;
      bool keep = false, gone = false;
      if (i < N) {
        // the whole slot in one batch of loads (a tombstone's other fields
        // are read but not used)
        wsk = P.sk[i];
        wes = P.es[i];
        wbb = P.bb[i];
        wpp = P.pp[i];
        if (bits(wsk.y) != kDead) {
          const bool stale = !idx_ok(c, wes.y, a.m.nv) || wsk.x > from_bits(lda(&a.s.g[wes.y]));
          if (stale) {
            stale_n++;
            gone = true;
          } else {
            have = tab ? (wsk.y <= cv) : (all || ((bits(wsk.y) >> sh) <= T));
            keep = !have;
          }
        }
      }
      if (have) n_sel++;
      if (inplace) {
        if (have || gone) reinterpret_cast<double*>(P.sk)[2 * i + 1] = from_bits(kDead);
        if (keep) kept_in++;
      } else {
        u64 jk, j1, j2;
        u32 tk, t1, t2;
        wave_reserve3(x.qctr, keep ? 1u : 0u, x.qctr, 0u, x.qctr, 0u, jk, j1, j2, tk, t1, t2);
        if (keep) {
          if (jk < (u64)a.cap)
            store_window(x.Q, jk, wbb.x, wbb.y, wpp.x, wpp.y, wsk.x, wsk.y, wes.x, wes.y);
          else
            flag_overflow(c);
        }
      }
      if (keep) {
        const u64 kb = bits(wsk.y);
        acc.kmn = kb < acc.kmn ? kb : acc.kmn;
        acc.kmx = kb > acc.kmx ? kb : acc.kmx;
      }
    } else {
      const u64 n = l_n[lvl];
      const u64 take = n < (u64)kBlock ? n : (u64)kBlock;
      have = threadIdx.x < take;
      if (have) {
        const u64 j = n - take + threadIdx.x;
        wbb = l_bb[lvl - 2][j];
        wpp = l_pp[lvl - 2][j];
        wsk = make_double2(l_sg[lvl - 2][j], 0.0);
        wes = l_es[lvl - 2][j];
      }
      __syncthreads();  // every thread has its window before the list shrinks
      if (threadIdx.x == 0) {
        l_n[lvl] = n - take;
        hopped += take;
      }
    }
    const int nl = lvl < kTop ? lvl + 1 : kTop;
    const HopList HQ{l_bb[nl - 2], l_pp[nl - 2], l_sg[nl - 2], l_es[nl - 2]};
    prop_window<true, HopList>(a, p, x, have, wbb, wpp, wsk, wes, lvl < hops, HQ, &l_n[nl], (u64)kFuseCap, acc);
    __syncthreads();  // the next list and its length are visible
    if (lvl < hops && l_n[lvl + 1] != 0) {
      ++lvl;
    } else {
      while (lvl > 1 && l_n[lvl] == 0) --lvl;
    }
  }
  u32 tot[3] = {stale_n, kept_in, n_sel};
  u64 z0 = kAllOnes, z1 = 0;
  block_totals(z0, z1, tot);
  if (threadIdx.x == 0) {
    if (tot[0] && a.counts) atomicAdd(&c->cnt[C_STALE], (u64)tot[0]);
    if (tot[1]) atomicAdd(&c->keptin, (u64)tot[1]);
    if (tot[2] + hopped) atomicAdd(&c->cnt[C_SEL], (u64)tot[2] + hopped);
    if (tot[2] && a.counts) atomicAdd(&c->xcnt[X_SEL1], (u64)tot[2]);
  }
  prop_finish(a, p, acc);
}

// Algorithm 4, first pass: geod_dist and the angle_split distance take the
// minimum over this round's events (keys: vertex, oriented edge).
// The lane's first distance event and first angle event, loaded together
// with the round's counters (indices below the capacities are in bounds).
struct FirstEvents {
  int2 vq;
  double d;
  double2 xy;
  int32_t e;
  double D, X;
};

__device__ __forceinline__ FirstEvents first_events(const RoundArgs& a, int p, u64 t0) {
  FirstEvents f{make_int2(0, -1), 0.0, make_double2(0.0, 0.0), 0, 0.0, 0.0};
  if (t0 < (u64)a.ecap) {
    f.vq = a.ev[p].vq[t0];
    f.d = a.ev[p].d[t0];
    f.xy = a.ev[p].xy[t0];
  }
  if (t0 < (u64)a.acap) {
    f.e = a.aev.e[t0];
    f.D = a.aev.D[t0];
    f.X = a.aev.X[t0];
  }
  return f;
}

// k_select_propagate with the first hopping child of every window kept in
// the lane's registers: only the second goes to the LDS list of the next hop,
// so a step adds at most one window per lane to a list and each list holds
// kBlock windows (12 KiB per hop level instead of 24 KiB), which leaves room
// for twice the workgroups per compute unit. A step at hop h propagates the
// register windows of hop h and, on the lanes without one, windows taken from
// the list of hop h; the steps go depth first as in k_propagate_fused (the
// deepest hop with work next), so when a step at hop h runs, the lists of the
// deeper hops are empty. The windows propagated at each hop, and every count,
// are those of the other launch plans.
// The workgroup (of BS threads) is thread t0 - threadIdx.x ... of the stride
// threads that share the round's scan: a whole launch, or the workgroups of
// a batched field's gang.
template <int NL, int BS>
__device__ __forceinline__ void ph_select_propagate(const RoundArgs& a, int p, u64 t0, u64 stride) {
  __shared__ double2 l_bb[NL][BS], l_pp[NL][BS];
  __shared__ double l_sg[NL][BS];
  __shared__ int2 l_es[NL][BS];
  __shared__ u64 l_n[NL + 2];  // l_n[h]: windows in the list of hop h (h >= 2)
  __shared__ u32 s_idle[BS / kWave];
  constexpr int kTop = NL + 1;  // the deepest hop
  Ctl* c = a.ctl;
  if (threadIdx.x <= (unsigned)kTop) l_n[threadIdx.x] = 0;
  const bool active = c->active != 0;
  const u64 pin = c->pin, pout = c->pout;
  const u64 N = active ? min(c->nscan, (u64)a.cap) : 0;
  const int sh = (int)c->shift;
  const u64 T = c->want;
  const bool all = c->sel_all;
  const bool tab = c->use_table;
  const double cv = c->cutval;
  const bool inplace = pin == pout;
  const Pool P = pin ? a.pool[1] : a.pool[0];
  const PropCtx x{pout ? a.pool[1] : a.pool[0], &c->npool[pout & 1], a.ev[p], sh, T, all, tab, cv};
  const int hops = a.hops < kTop ? a.hops : kTop;
  const int w = threadIdx.x / kWave, lane = lane_id();
  __syncthreads();
  PropAcc acc;
  RegWin rw;
  u32 stale_n = 0, kept_in = 0, n_sel = 0, n_hop = 0;
  __shared__ u32 s_ticket;
  bool first = true;
  u32 ticket = (u32)(t0 / BS);  // the workgroup's deal of the pool (scan_ticket)
  int lvl = 1;                  // hop of the next step (the same in every thread)
  for (;;) {
    bool have = false;
    double2 wbb = make_double2(0.0, 0.0), wpp = wbb, wsk = wbb;
    int2 wes = make_int2(0, 0);
    u64 rest = 0;  // the length of this hop's list after the step (hops >= 2)
    if (lvl == 1) {
      u64 i = 0;
      if (!scan_ticket(c, N, (u32)(stride / BS), BS / kWave, first, ticket, &s_ticket, i)) break;
      bool keep = false, gone = false;
      if (i < N) {
        wsk = P.sk[i];
        wes = P.es[i];
        wbb = P.bb[i];
        wpp = P.pp[i];
        if (bits(wsk.y) != kDead) {
          const bool stale = !idx_ok(c, wes.y, a.m.nv) || wsk.x > from_bits(lda(&a.s.g[wes.y]));
          if (stale) {
            stale_n++;
            gone = true;
          } else {
            have = tab ? (wsk.y <= cv) : (all || ((bits(wsk.y) >> sh) <= T));
            keep = !have;
          }
        }
      }
      if (have) n_sel++;
      if (inplace) {
        if (have || gone) reinterpret_cast<double*>(P.sk)[2 * i + 1] = from_bits(kDead);
        if (keep) kept_in++;
      } else {
        u64 jk, j1, j2;
        u32 tk, t1, t2;
        wave_reserve3(x.qctr, keep ? 1u : 0u, x.qctr, 0u, x.qctr, 0u, jk, j1, j2, tk, t1, t2);
        if (keep) {
          if (jk < (u64)a.cap)
            store_window(x.Q, jk, wbb.x, wbb.y, wpp.x, wpp.y, wsk.x, wsk.y, wes.x, wes.y);
          else
            flag_overflow(c);
        }
      }
      if (keep) {
        const u64 kb = bits(wsk.y);
        acc.kmn = kb < acc.kmn ? kb : acc.kmn;
        acc.kmx = kb > acc.kmx ? kb : acc.kmx;
      }
    } else {
      // the lane's register window of this hop, else one from the list: the
      // lanes without a register window are ranked and take the list's last
      // windows in rank order (s_idle, each wavefront's count of such lanes,
      // was written before the barrier that ended the previous step)
      const bool idle = !rw.has;
      const u64 m = __ballot(idle);
      const u32 wrank = (u32)__popcll(m & ((1ull << lane) - 1ull));
      u32 rank = wrank;
      for (int q = 0; q < w; ++q) rank += s_idle[q];
      u32 n_idle = 0;
      for (int q = 0; q < BS / kWave; ++q) n_idle += s_idle[q];
      const u64 n = l_n[lvl];
      const u64 take = n < (u64)n_idle ? n : (u64)n_idle;
      if (!idle) {
        have = true;
        wbb = rw.bb;
        wpp = rw.pp;
        wsk = make_double2(rw.sg, 0.0);
        wes = rw.es;
      } else if (rank < take) {
        const u64 j = n - take + rank;
        have = true;
        wbb = l_bb[lvl - 2][j];
        wpp = l_pp[lvl - 2][j];
        wsk = make_double2(l_sg[lvl - 2][j], 0.0);
        wes = l_es[lvl - 2][j];
      }
      rest = n - take;
      if (have) n_hop++;
    }
    const int nl = lvl < kTop ? lvl + 1 : kTop;
    const HopList HQ{l_bb[nl - 2], l_pp[nl - 2], l_sg[nl - 2], l_es[nl - 2]};
    prop_window<true, HopList, true, BS>(a, p, x, have, wbb, wpp, wsk, wes, lvl < hops, HQ, &l_n[nl], (u64)BS,
                                         acc, &rw);
    // The list of this hop shrinks only now: every thread read its length
    // before the reservation barriers of prop_window, and no thread appends
    // to it in this step (children go to the list of the next hop; the last
    // hop appends nothing), so its windows taken above stay intact.
    if (lvl >= 2 && threadIdx.x == 0) l_n[lvl] = rest;
    // the lanes without a register window, for the next step's ranking (every
    // thread read the previous counts before the reservation barriers)
    const u64 idle_next = __ballot(!rw.has);
    if (lane == 0) s_idle[w] = (u32)__popcll(idle_next);
    // deeper when some lane holds a register window or the next list has
    // windows (the list length is visible after the barrier)
    const int deeper = __syncthreads_or(rw.has ? 1 : 0);
    if (lvl < hops && (deeper || l_n[lvl + 1] != 0)) {
      ++lvl;
    } else {
      while (lvl > 1 && l_n[lvl] == 0) --lvl;
    }
  }
  u32 tot[4] = {stale_n, kept_in, n_sel, n_hop};
  u64 z0 = kAllOnes, z1 = 0;
  block_totals(z0, z1, tot);
  if (threadIdx.x == 0) {
    if (tot[0] && a.counts) atomicAdd(&c->cnt[C_STALE], (u64)tot[0]);
    if (tot[1]) atomicAdd(&c->keptin, (u64)tot[1]);
    if (tot[2] + tot[3]) atomicAdd(&c->cnt[C_SEL], (u64)tot[2] + tot[3]);
    if (tot[2] && a.counts) atomicAdd(&c->xcnt[X_SEL1], (u64)tot[2]);
  }
  prop_finish(a, p, acc);
}

// Three workgroups per compute unit hold the four hop lists of the 5-hop
// instance in LDS; the bound keeps the registers within a third of the file
// (at most 168 per lane) so that the registers allow three as well.
template <int NL>
__global__ void __launch_bounds__(kBlock, 3) k_select_propagate_r(RoundArgs a, int p) {
  ph_select_propagate<NL, kBlock>(a, p, blockIdx.x * (u64)kBlock + threadIdx.x, (u64)gridDim.x * kBlock);
}

// Algorithm 4, first event pass (the minima themselves were taken by the
// propagation and the previous round's fans, in geod_dist's and
// angle_split's write copies): each corner keeps the smallest crossing among
// the angle events that reached its (new or unchanged) apex distance,
// together with a kept old crossing: the lexicographic minimum of (distance,
// crossing). An event that reached its vertex's new distance copies it into
// geod_dist, and each improved pseudo-source vertex records the smallest
// incoming angle among those events.
// A winning event at a pseudo-source vertex goes to the fan pass's candidate
// list, one reservation per wavefront (every lane of the wavefront calls it),
// or with kBlk one per workgroup (every thread of the workgroup calls it).
template <bool kBlk = false>
__device__ __forceinline__ void add_candidate(const RoundArgs& a, Ctl* c, bool win, int32_t v, double d) {
  if constexpr (kBlk) {
    u64 j, s1, s2, s3;
    u32 t0, t1, t2, t3;
    block_reserve4(&c->ncand, win ? 1u : 0u, &c->ncand, 0u, &c->ncand, 0u, &c->ncand, 0u, j, s1, s2, s3, t0, t1, t2,
                   t3);
    if (win && j < (u64)a.ecap) {
      a.cand.vq[j] = make_int2(v, -1);
      a.cand.d[j] = d;
    }
    return;
  }
  const u64 mask = __ballot(win);
  if (!mask) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  u64 base = 0;
  if (lane_id() == leader) base = atomicAdd(&c->ncand, (u64)__popcll(mask));
  base = shfl64(base, leader);
  if (win) {
    const u64 j = base + (u64)__popcll(mask & ((1ull << lane_id()) - 1ull));
    if (j < (u64)a.ecap) {
      a.cand.vq[j] = make_int2(v, -1);
      a.cand.d[j] = d;
    }
  }
}

template <bool kBlk = false>
__device__ __forceinline__ void ph_events2(const RoundArgs& a, int p, u64 t0, u64 stride) {
  Ctl* c = a.ctl;
  const FirstEvents f = first_events(a, p, t0);
  const bool active = c->active != 0;
  const u64 nd = active ? min(c->ndev[p], (u64)a.ecap) : 0;
  const u64 na = active ? min(c->naev, (u64)a.acap) : 0;
  const u32 stamp = (u32)c->round;
  // The lane's first angle event and first distance event take every load
  // that depends only on their records in one batch: the corner's apex
  // distance, the vertex's write-copy distance and flags, and the half-edge
  // values of the incoming-angle recipe (an event with a recipe names a
  // pseudo-source vertex; the angle is evaluated for the winners only).
  const bool aok = t0 < na && idx_ok(c, f.e, a.m.nh);
  const bool vok = t0 < nd && idx_ok(c, f.vq.x, a.m.nv);
  const bool rok = vok && f.vq.y >= 0 && idx_ok(c, f.vq.y >> 2, a.m.nh);
  const int32_t ea = aok ? f.e : 0;
  const int32_t v = vok ? f.vq.x : 0;
  const u64 asD = lda(&a.s.asw[ea].D);
  const u64 gwv = lda(&a.s.gw[v]);
  const uint8_t fl = a.m.flags[v];
  const AngleRecipe rc = load_recipe(a.m, rok ? f.vq.y : 0);
  if (aok && bits(f.D) == asD) atomicMin(&a.s.asw[ea].X, ordkey(f.X));
  {
    const bool top = vok && bits(f.d) == gwv;
    if (top) a.s.g[v] = bits(f.d);
    const bool win = top && (fl & pch::VF_PSEUDO);
    double th = 0.0;
    bool first = false;
    if (win) {
      // the first winner to claim a pseudo-source vertex this round lists it
      // for its fan (the claim is issued first, so that its round trip
      // overlaps the evaluation of the winner's incoming angle)
      const u32 old = atomicMax(&a.s.claim[v], stamp);
      th = f.vq.y >= 0 ? recipe_angle(rc, f.xy.x, f.xy.y) : f.xy.x;
      atomicMin(&a.s.fanth[v], ordkey(th));
      first = old < stamp;
    }
    add_candidate<kBlk>(a, c, first, v, f.d);
  }
  // the rest (more events than the launch has threads)
  for (u64 i = t0 + stride; i < na; i += stride) {
    const int32_t e = a.aev.e[i];
    const double D = a.aev.D[i];
    const double X = a.aev.X[i];
    if (idx_ok(c, e, a.m.nh) && bits(D) == lda(&a.s.asw[e].D)) atomicMin(&a.s.asw[e].X, ordkey(X));
  }
  // (wave-uniform trip count; workgroup-uniform with kBlk)
  for (u64 i = t0 + stride; i - (kBlk ? threadIdx.x : lane_id()) < nd; i += stride) {
    bool win = false;
    int32_t vi = 0;
    double d = 0.0, th = 0.0;
    if (i < nd) {
      const int2 vq = a.ev[p].vq[i];
      d = a.ev[p].d[i];
      const double2 xy = a.ev[p].xy[i];
      vi = vq.x;
      const bool top = idx_ok(c, vi, a.m.nv) && bits(d) == lda(&a.s.gw[vi]);
      if (top) a.s.g[vi] = bits(d);
      if (top && (a.m.flags[vi] & pch::VF_PSEUDO)) {
        const u32 old = atomicMax(&a.s.claim[vi], stamp);
        th = vq.y >= 0 ? event_angle(a.m, vq.y, xy.x, xy.y) : xy.x;
        atomicMin(&a.s.fanth[vi], ordkey(th));
        win = old < stamp;
      }
    }
    add_candidate<kBlk>(a, c, win, vi, d);
  }
}

__global__ void __launch_bounds__(kBlock) k_events2(RoundArgs a, int p) {
  ph_events2<true>(a, p, blockIdx.x * (u64)kBlock + threadIdx.x, (u64)gridDim.x * kBlock);
}

// Second event pass: the corners' final values into angle_split, and one fan
// per improved pseudo-source vertex: windows into the next pool, deferred
// endpoint events into geod_dist's write copy and the next round's event
// buffer.
template <bool kBlk = false>
__device__ __forceinline__ void ph_events3(const RoundArgs& a, int p, u64 t0, u64 stride) {
  Ctl* c = a.ctl;
  // Distance events are dealt round-robin over the launch's wavefronts (event
  // w + nw * lane of each stride-wide chunk to lane `lane` of wavefront w), so
  // the few fans of a round spread over many compute units.
  const u64 nw = stride / kWave, w = t0 / kWave;
  const u64 i0 = w + nw * (u64)lane_id();
  // the lane's first candidate is loaded together with the round's counters
  // (indices below the capacity are in bounds)
  int32_t f_v = 0;
  double f_d = 0.0;
  if (i0 < (u64)a.ecap) {
    f_v = a.cand.vq[i0].x;
    f_d = a.cand.d[i0];
  }
  int32_t f_e = 0;
  if (t0 < (u64)a.acap) f_e = a.aev.e[t0];
  const bool active = c->active != 0;
  const u64 nd = active ? min(c->ncand, (u64)a.ecap) : 0;
  const u64 na = active ? min(c->naev, (u64)a.acap) : 0;
  const int po = (int)(c->pout & 1);
  // the corners this round's angle events touched take their final values
  // (the first event pass is over) from the write copy; the lane's first
  // corner is copied together with its first candidate's loads below (the
  // fans neither read nor write angle_split)
  const bool f_ok = t0 < na && idx_ok(c, f_e, a.m.nh);
  u64 f_swD = 0, f_swX = 0;  // the corner's write copy, stored after the fans
  if (f_ok) {
    f_swD = a.s.asw[f_e].D;
    f_swX = a.s.asw[f_e].X;
  }
  for (u64 i = t0 + stride; i < na; i += stride) {
    const int32_t e = a.aev.e[i];
    if (idx_ok(c, e, a.m.nh)) a.s.as[e] = a.s.asw[e];
  }
  u64 kmn = kAllOnes, kmx = 0;
  u32 kept = 0, tiny = 0, ich = 0, defer = 0, notwin = 0, fans = 0;
  // (wave-uniform trip count; workgroup-uniform with kBlk)
  const u64 wl = kBlk ? (t0 - threadIdx.x) / kWave : w;
  for (u64 j0 = 0; wl + j0 < nd; j0 += stride) {
    const u64 i = j0 + i0;
    bool has = false;
    int v = 0, q0 = 0, q1 = 0;
    double d = 0.0, th = 0.0;
    if (i < nd) {
      if (j0 == 0) {
        v = f_v;
        d = f_d;
      } else {
        v = a.cand.vq[i].x;
        d = a.cand.d[i];
      }
      const bool okv = idx_ok(c, v, a.m.nv);
      if (!okv) v = 0;
      // a candidate is a vertex that a winning event reached at a
      // pseudo-source, listed once (claimed in the first pass); its fan starts
      // from the round's distance with the smallest incoming angle of its
      // winners
      const u64 fv = lda(&a.s.fanth[v]);
      q0 = a.m.coff[v];
      q1 = a.m.coff[v + 1];
      if (okv) {
        a.s.fanth[v] = kAllOnes;
        th = from_ordkey(fv);
        has = true;
        fans++;
      }
    }
    wave_fans<kBlk>(a, has, v, q0, q1 - q0, d, th, a.full_fan != 0, po, 1 - p, kmn, kmx, kept, tiny, ich, defer,
                    notwin);
  }
  if (f_ok) {
    a.s.as[f_e].D = f_swD;
    a.s.as[f_e].X = f_swX;
  }
  u32 tot[5] = {kept, tiny, ich, fans, notwin};
  block_totals(kmn, kmx, tot);
  if (threadIdx.x == 0) {
    if (kmn != kAllOnes) atomicMin(&c->kmin[1 - p], kmn);
    if (kmx != 0) atomicMax(&c->kmax[1 - p], kmx);
    if (a.counts) {
      if (tot[0]) atomicAdd(&c->cnt[C_FANWIN], (u64)tot[0]);
      if (tot[1]) atomicAdd(&c->cnt[C_TINY], (u64)tot[1]);
      if (tot[2]) atomicAdd(&c->cnt[C_ICH], (u64)tot[2]);
      if (tot[3]) atomicAdd(&c->cnt[C_FANS], (u64)tot[3]);
      if (tot[4]) atomicAdd(&c->xcnt[X_NOTWIN], (u64)tot[4]);
    }
  }
}

// The last block to finish sets up the next round.
__global__ void __launch_bounds__(kBlock) k_events3(RoundArgs a, int p) {
  __shared__ int is_last;
  Ctl* c = a.ctl;
  ph_events3<true>(a, p, blockIdx.x * (u64)kBlock + threadIdx.x, (u64)gridDim.x * kBlock);
  // The set-up reads only counters, which every workgroup updates with
  // device-scope atomics and the set-up reads with device-scope atomic loads;
  // waiting until this wavefront's memory operations have completed orders
  // its counter updates before the ticket. (A device-scope fence would also
  // write back the L2 caches, which the set-up does not need: it reads no
  // plain stores of this kernel.)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(&c->ticket, 1ull) == (u64)(gridDim.x - 1);
  __syncthreads();
  if (is_last && threadIdx.x < kWave) {
    if (threadIdx.x == 0) c->ticket = 0;
    round_begin(a, 1 - p);
  }
}


// ---------------------------------------------------------------------------
// batched fields: one workgroup runs every round of one field at a time
// ---------------------------------------------------------------------------

struct alignas(256) GangRec;

struct BatchDev {
  const DevMesh* meshes;      // [n_meshes]
  const int64_t* mesh_nv;     // [n_meshes]
  const int64_t* mesh_nh;     // [n_meshes]
  const double* mesh_delta0;  // [n_meshes] first adaptive step
  const int32_t* field_mesh;  // [n_fields]
  const int32_t* field_src;   // [n_fields]
  const int64_t* field_off;   // [n_fields] offset of the field in out
  const int32_t* order;       // [n_fields] processing order (largest cost first)
  const u64* cost;            // [n_fields] expected workgroup time of the field (any unit)
  const u64* wins;            // [n_fields] expected windows of the field
  int32_t n_fields;           // fields taken from the queue
  double* out;                // concatenated distance fields
  int64_t* fstat;             // [n_fields][kFieldStat]
  u64* queue;                 // [2]: next position in order, fields taken but not yet offered
  GangRec* gang;              // [n_fields] round handshake of the field's workgroups
  u32* board;                 // [kMaxXcc][kBoard] field + 1 of a running field that takes helpers, or 0
  // per-team buffers (team t uses slot t)
  double2 *pbb, *ppp, *psk;  // [n_teams][nslot][cap]: pool 0, pool 1, selection, hop queues
  int2* pes;
  int2* ev_vq;  // [n_teams][3][ecap]: events of parity 0 and 1, fan candidates
  double* ev_d;
  double2* ev_xy;
  int32_t* ae_e;  // [n_teams][acap]
  double *ae_D, *ae_X;
  u64 *g, *gw, *fanth;  // [n_teams][max_nv]
  u32* claim;           // [n_teams][max_nv]
  Split *as, *asw;      // [n_teams][max_nh]
  int64_t cap, ecap, acap, max_nv, max_nh;
  int64_t k;
  double eps;
  int32_t ch_on, ich_on, full_fan, retest;
  int32_t hops;      // propagation hops per round
  int32_t nslot;     // window buffers per team: pool 0, pool 1, selection (+ 2 hop queues)
  int32_t gang_max;  // workgroups per field (1: no helpers)
  int32_t n_store;   // workgroups with buffers of their own; the others only help
  u64 wait;          // longest wait of a gang member, wall-clock ticks
  int64_t max_rounds;
  int32_t mode;       // PCH_SELECT_DELTA or PCH_SELECT_LEARNED
  const u32* cdf;     // LEARNED: [n_fields][kCdfBins + 1] predicted-distance tables
  const double* pbin; // LEARNED: [n_fields] bin widths
  double w0;
};

// status, rounds, processed, created, fans, peak pool, stale, leader time,
// helpers, helper time
constexpr int kFieldStat = 10;
constexpr int kMaxXcc = 16;    // XCD ids covered by the board
constexpr int kBoard = 64;     // running fields per XCD that helpers can find
constexpr int kMaxGang = 32;   // workgroups on one field
// Default longest wait of a gang member for the others, in ticks of the
// 100 MHz wall clock (2 s): far above any round, so it only ends a wait that
// cannot end.
constexpr u64 kGangWait = 200000000ull;
// Status of a batched field (the first field_stats column). The host reruns
// every field whose status is not PCH_FIELD_OK through pch_geodesic with the
// same rule, which either finishes it (a larger pool, no gang) or returns the
// error (non-finite geometry, an index outside the mesh).
__host__ __device__ __forceinline__ int64_t field_status(bool ok, bool overflow, bool over_rounds, bool nonfinite,
                                                         bool badidx) {
  if (badidx) return PCH_FIELD_BAD_INDEX;
  if (nonfinite) return PCH_FIELD_NONFINITE;
  if (!ok) return PCH_FIELD_ABANDONED;
  if (overflow) return PCH_FIELD_OVERFLOW;
  if (over_rounds) return PCH_FIELD_MAX_ROUNDS;
  return PCH_FIELD_OK;
}
// field status before a workgroup finishes it
constexpr int64_t kFieldNotRun = PCH_FIELD_NOT_RUN;

// The workgroups that share one field: the leader (the workgroup that took
// the field, whose buffers hold it) and the helpers of the same XCD that
// joined it between rounds. All of them reach the field's buffers through the
// one L2 of their XCD.
struct alignas(256) GangRec {
  u64 word;   // round handshake: (count << 8) | (done << 7) | (parity << 6) | members
  u64 join;   // helpers that joined
  u64 left;   // helpers that left
  u64 abort;  // 1 after a member's wait ran out of time
  u64 team;   // the leader's workgroup
  u64 prog;   // windows processed so far (published by the leader each round)
  u64 hticks; // wall-clock ticks the helpers spent in the field
  u64 pad0[9];
  u64 cnt[2];  // barrier arrivals in rounds of even and odd count
  u64 pad1[14];
  Ctl ctl;  // round counters from the first round with helpers on
};

// Barrier between the phases of a field that one workgroup runs alone: the
// workgroup's wavefronts share the compute unit's L1 and its in-order vector
// memory pipeline, so a plain workgroup barrier orders one phase's stores and
// atomics before the next phase's loads. A device-scope fence would also
// write back the L2 cache at every phase.
__device__ __forceinline__ void team_sync() { __syncthreads(); }

__device__ __forceinline__ void sta(u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the XCD (accelerator complex die) this wavefront runs on
__device__ __forceinline__ u32 xcc_id() {
  u32 x;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
  return x & 0xfu;
}
// Agent-scope acquire: drops the compute unit's vector L1 lines (buffer_inv
// sc1), so that later plain loads see what other compute units stored. The
// workgroup-scope invalidate (sc0) leaves those lines in place on gfx950: a
// reader on another compute unit of the same XCD kept reading its stale
// copies after it.
__device__ __forceinline__ void l1_invalidate() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Barrier of the nm workgroups of a gang round. Every wavefront first waits
// for its own stores and atomics (they are then in the XCD's L2, which every
// member reads through), one lane per workgroup arrives, and after the wait
// the compute unit's L1 is dropped, so that the next phase's plain loads (the
// round counters included) see what the other members stored and updated
// atomically. Returns 0 when the gang gave up: some member's wait ran out of
// time, which sets the gang's abort flag for all of them.
__device__ __forceinline__ int gang_sync(GangRec* R, int slot, u64 target, u64 wait, int* s_ok) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&R->cnt[slot], 1ull);
    int ok = 1;
    const u64 t_end = wall_clock64() + wait;
    while (ld(&R->cnt[slot]) < target) {
      if (ld(&R->abort) || wall_clock64() > t_end) {
        sta(&R->abort, 1ull);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    l1_invalidate();
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok;
}

__device__ __forceinline__ Pool slot_pool(const BatchDev& B, int t, int b) {
  const int64_t o = ((int64_t)t * B.nslot + b) * B.cap;
  return Pool{B.pbb + o, B.ppp + o, B.psk + o, B.pes + o};
}

// Round arguments of field f in the buffers of workgroup t (without the
// control block), written straight into the workgroup's LDS copy.
__device__ __forceinline__ void team_args(const BatchDev& B, int t, int f, RoundArgs& a) {
  const int mi = B.field_mesh[f];
  a.m = B.meshes[mi];
  a.s = DevState{B.g + t * B.max_nv,     B.as + t * B.max_nh,  B.fanth + t * B.max_nv,
                 B.claim + t * B.max_nv, B.gw + t * B.max_nv, B.asw + t * B.max_nh};
  a.pool[0] = slot_pool(B, t, 0);
  a.pool[1] = slot_pool(B, t, 1);
  a.sel = slot_pool(B, t, 2);
  a.hq[0] = B.hops > 1 ? slot_pool(B, t, 3) : Pool{};
  a.hq[1] = B.hops > 1 ? slot_pool(B, t, 4) : Pool{};
  a.hops = B.hops;
  a.org_shift = -1;  // batched fields are not organized by edge
  a.sorted = Pool{};
  a.org_hist = nullptr;
  a.org_ofs = nullptr;
  for (int i = 0; i < 2; ++i) {
    const int64_t o = ((int64_t)t * 3 + i) * B.ecap;
    a.ev[i] = DistEv{B.ev_vq + o, B.ev_d + o, B.ev_xy + o};
  }
  const int64_t oc = ((int64_t)t * 3 + 2) * B.ecap;
  a.cand = DistEv{B.ev_vq + oc, B.ev_d + oc, B.ev_xy + oc};
  const int64_t oa = (int64_t)t * B.acap;
  a.aev = AngEv{B.ae_e + oa, B.ae_D + oa, B.ae_X + oa};
  a.ctl = nullptr;
  a.hist = nullptr;
  a.log = nullptr;
  a.max_log = 0;
  a.cap = B.cap;
  a.ecap = B.ecap;
  a.acap = B.acap;
  a.k = B.k;
  a.mode = B.mode;
  a.eps = B.eps;
  a.ch_on = B.ch_on;
  a.ich_on = B.ich_on;
  a.full_fan = B.full_fan;
  a.retest = B.retest;
  a.table = nullptr;
  a.n_table = 0;
  const bool learned = B.mode == PCH_SELECT_LEARNED;
  a.cdf = learned ? B.cdf + (int64_t)f * (kCdfBins + 1) : nullptr;
  a.pbin = learned ? B.pbin[f] : 0.0;
  a.w0 = B.w0;
  a.counts = 1;
}

// Out-of-line phases for the persistent kernel: each gets its own register
// allocation instead of the union of all phases in one function.
__device__ __noinline__ void nl_partition(const RoundArgs& a, int p, u64 t0, u64 s) { ph_partition(a, p, t0, s); }
__device__ __noinline__ void nl_propagate(const RoundArgs& a, int p, int hop, u64 t0, u64 s) {
  ph_propagate(a, p, hop, t0, s);
}
__device__ __noinline__ void nl_events2(const RoundArgs& a, int p, u64 t0, u64 s) { ph_events2(a, p, t0, s); }
__device__ __noinline__ void nl_events3(const RoundArgs& a, int p, u64 t0, u64 s) { ph_events3(a, p, t0, s); }
__device__ __noinline__ void nl_begin(const RoundArgs& a, int p) { round_begin(a, p); }
__device__ __forceinline__ void init_fan(const RoundArgs& a, int v, Ctl* ctl) {
  u64 kmn = kAllOnes, kmx = 0;
  u32 kept = 0, tiny = 0, ich = 0, defer = 0, notwin = 0;
  const int q0 = a.m.coff[v];
  wave_fans(a, lane_id() == 0, v, q0, a.m.coff[v + 1] - q0, 0.0, 0.0, true, 0, 0, kmn, kmx, kept, tiny, ich,
            defer, notwin);
  kmn = wave_min64(kmn);
  kmx = wave_max64(kmx);
  if (lane_id() == 0) {
    if (kmn != kAllOnes) atomicMin(&ctl->kmin[0], kmn);
    if (kmx != 0) atomicMax(&ctl->kmax[0], kmx);
  }
}
__device__ __noinline__ void nl_init_fan(const RoundArgs& a, int v, Ctl* ctl) { init_fan(a, v, ctl); }

// Phases of the persistent kernel: 1024-thread teams (at most 128 VGPRs per
// lane) call them out of line, each with its own register allocation;
// 256- and 512-thread teams (up to 512 and 256 VGPRs) inline them into one
// allocation without spills.
template <bool kOOL>
struct TeamPhases {
  static __device__ __forceinline__ void init_fan_(const RoundArgs& a, int v, Ctl* ctl) {
    if constexpr (kOOL) nl_init_fan(a, v, ctl); else init_fan(a, v, ctl);
  }
  static __device__ __forceinline__ void begin(const RoundArgs& a, int p) {
    if constexpr (kOOL) nl_begin(a, p); else round_begin(a, p);
  }
  static __device__ __forceinline__ void partition(const RoundArgs& a, int p, u64 t0, u64 s) {
    if constexpr (kOOL) nl_partition(a, p, t0, s); else ph_partition(a, p, t0, s);
  }
  static __device__ __forceinline__ void propagate(const RoundArgs& a, int p, int hop, u64 t0, u64 s) {
    if constexpr (kOOL) nl_propagate(a, p, hop, t0, s); else ph_propagate(a, p, hop, t0, s);
  }
  static __device__ __forceinline__ void events2(const RoundArgs& a, int p, u64 t0, u64 s) {
    if constexpr (kOOL) nl_events2(a, p, t0, s); else ph_events2(a, p, t0, s);
  }
  static __device__ __forceinline__ void events3(const RoundArgs& a, int p, u64 t0, u64 s) {
    if constexpr (kOOL) nl_events3(a, p, t0, s); else ph_events3(a, p, t0, s);
  }
};

// The phases of one round (Algorithm 1) as member idx of nm workgroups: the
// member's threads take every nm-th block of the work. With one member the
// phases are separated by workgroup barriers, otherwise by gang barriers on
// arrival counter `slot`. Returns 0 when the gang gave up.
template <class Ph, int BS>
__device__ __forceinline__ int team_round(const RoundArgs& a, int p, int idx, int nm, GangRec* R, int slot, u64 wait,
                                          int* s_ok) {
  const u64 t0 = (u64)idx * BS + threadIdx.x, stride = (u64)nm * BS;
  u64 nb = 0;
  auto bar = [&]() -> int {
    if (nm == 1) {
      team_sync();
      return 1;
    }
    return gang_sync(R, slot, (u64)nm * ++nb, wait, s_ok);
  };
  Ph::partition(a, p, t0, stride);
  if (!bar()) return 0;
  Ph::propagate(a, p, 1, t0, stride);
  if (!bar()) return 0;
  for (int h = 2; h <= a.hops; ++h) {
    if (ld(&a.ctl->nhop[h - 1]) == 0) break;
    Ph::propagate(a, p, h, t0, stride);
    if (!bar()) return 0;
  }
  Ph::events2(a, p, t0, stride);
  if (!bar()) return 0;
  Ph::events3(a, p, t0, stride);
  return bar();
}

// A helper's share of gang R as member idx: between rounds it waits for the
// leader's handshake, which names the round's parity and member count and
// whether the field is finished.
template <class Ph, int BS>
__device__ __forceinline__ void help_field(const BatchDev& B, GangRec* R, int idx, RoundArgs& sa, int* s_ok, u64* s_word) {
  const u64 t_join = wall_clock64();
  if (threadIdx.x == 0) {
    team_args(B, (int)ld(&R->team), (int)(R - B.gang), sa);
    sa.ctl = &R->ctl;
  }
  u64 seen = 0;
  for (;;) {
    __syncthreads();  // every wavefront has read the previous handshake
    if (threadIdx.x == 0) {
      const u64 t_end = wall_clock64() + B.wait;
      u64 w;
      for (;;) {
        w = ld(&R->word);
        if (w != seen) break;
        if (ld(&R->abort) || wall_clock64() > t_end) {
          sta(&R->abort, 1ull);
          w = 1ull << 7;  // treat as finished
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      l1_invalidate();
      *s_word = w;
    }
    __syncthreads();
    const u64 w = *s_word;
    if (w & (1ull << 7)) break;
    seen = w;
    const int nm = (int)(w & 63);
    if (idx >= nm) continue;
    if (!team_round<Ph, BS>(sa, (int)((w >> 6) & 1), idx, nm, R, (int)((w >> 8) & 1), B.wait, s_ok)) break;
  }
  if (threadIdx.x == 0) {
    atomicAdd(&R->hticks, wall_clock64() - t_join);
    __builtin_amdgcn_s_waitcnt(0);
    atomicAdd(&R->left, 1ull);
  }
  __syncthreads();
}

// Persistent workgroups: each takes the next field from the queue and runs
// Algorithm 1 on it, the phases separated by workgroup barriers and the round
// counters in LDS; fields never wait for each other. A field that outgrows
// the team's pool is flagged for a rerun by the host. With gang_max > 1 a
// running field accepts helpers: a free workgroup joins a running field of
// its own XCD when that field's expected time left per member exceeds the
// next queued field's (or the queue is empty), and from the next round on the
// field's rounds are split over its members (the counters then live in the
// field's gang record).
template <int BS>
__global__ void __launch_bounds__(BS) k_batch(BatchDev B) {
  using Ph = TeamPhases<(BS > 512)>;
  __shared__ Ctl lctl;
  __shared__ RoundArgs sa;
  __shared__ int cur, s_ok, s_nm, s_slot, s_done, s_stop, s_pick, s_idx;
  __shared__ u64 s_word;
  const int t = blockIdx.x;
  const u64 t0 = threadIdx.x, stride = BS;
  const u32 xcc = xcc_id();
  const bool gangs = B.gang_max > 1 && xcc < (u32)kMaxXcc;
  u32* board = B.board + (size_t)(xcc < (u32)kMaxXcc ? xcc : 0) * kBoard;
  int fails = 0, idle = 0;
  if (gangs) {
    // Stagger the first choice (about 0.8 us per eight workgroups), so that
    // the leaders of the first fields have offered them when the later
    // workgroups choose between joining one and taking the next field.
    for (int i = 0; i < (t >> 3); ++i) __builtin_amdgcn_s_sleep(30);
  }
  for (;;) {
    // Next work: the next field of the queue (longest expected first), or a
    // running field of this XCD whose remaining windows per workgroup, with
    // this one joined, exceed the next queued field's.
    __syncthreads();  // every wavefront has read the previous choice
    if (threadIdx.x < (u32)kWave) {
      u64 key = 0;  // (remaining windows per member << 32) | ~field
      if (gangs) {
        // lane l looks at board entry l
        const u32 e = lane_id() < kBoard ? __hip_atomic_load(&board[lane_id()], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT) : 0u;
        if (e != 0u) {
          GangRec* Rc = B.gang + (e - 1u);
          const u64 j = ld(&Rc->join);
          if (j < (u64)(B.gang_max - 1) && !(ld(&Rc->word) & (1ull << 7))) {
            // expected time left: the cost times the share of its windows
            // not processed yet
            const u64 wf = B.wins[e - 1u], pr = ld(&Rc->prog);
            const double left = wf > pr ? (double)(wf - pr) / (double)wf : 0.0;
            const u64 rem = (u64)((double)B.cost[e - 1u] * left) + 1;
            key = (min(rem / (j + 2), (u64)0xffffffffu) << 32) | (u64)(0xffffffffu - (e - 1u));
          }
        }
        key = wave_max64(key);
      }
      if (threadIdx.x == 0) {
        // >= 0: help that field; -1: no work left; -2: look again; -3: lead
        // `cur`; -4: a field is queued or about to be offered, and only a
        // workgroup with buffers may lead it
        int pick = -1;
        const u64 q = ld(B.queue);
        const bool queued = q < (u64)B.n_fields;
        const u64 cq = queued ? B.cost[B.order[q]] : 0;
        if (key != 0 && (!queued || (key >> 32) > cq)) {
          const u32 f = 0xffffffffu - (u32)key;
          GangRec* Rc = B.gang + f;
          const u64 j = ld(&Rc->join);
          pick = -2;  // the field changed meanwhile
          if (j < (u64)(B.gang_max - 1) && atomicCAS(&Rc->join, j, j + 1) == j) {
            pick = (int)f;
            s_idx = (int)j + 1;
          }
        } else if (queued && t >= B.n_store) {
          pick = -4;  // no buffers of its own: wait for a field to share
        } else if (queued) {
          const u64 q2 = atomicAdd(B.queue, 1ull);
          pick = -2;  // the queue ran out meanwhile
          if (q2 < (u64)B.n_fields) {
            cur = B.order[q2];
            pick = -3;
          }
        } else if (gangs && ld(B.queue + 1) > 0) {
          pick = -4;
        }
        if (pick == -3 && gangs) atomicAdd(B.queue + 1, 1ull);
        s_pick = pick;
      }
    }
    __syncthreads();
    const int pick = s_pick;
    if (pick == -1) return;
    if (pick == -2) {
      if (++fails > 4096) return;
      continue;
    }
    if (pick == -4) {
      // about 3.4 us per look; stop looking after about 2 s without work
      if (++idle > 600000) return;
      __builtin_amdgcn_s_sleep(127);
      continue;
    }
    fails = 0;
    idle = 0;
    if (pick >= 0) {
      help_field<Ph, BS>(B, B.gang + pick, s_idx, sa, &s_ok, &s_word);
      continue;
    }
    const int f = cur;
    const u64 t_start = wall_clock64();
    const int mi = B.field_mesh[f];
    const int64_t nv = B.mesh_nv[mi], nh = B.mesh_nh[mi];
    GangRec* R = gangs ? B.gang + f : nullptr;
    if (threadIdx.x == 0) {
      team_args(B, t, f, sa);
      sa.ctl = &lctl;
      // zero the control block
      u64* cw = (u64*)&lctl;
      for (size_t w = 0; w < sizeof(Ctl) / sizeof(u64); ++w) cw[w] = 0;
      lctl.kmin[0] = lctl.kmin[1] = kAllOnes;
      lctl.delta = B.mesh_delta0[mi];
      lctl.lfac = 1.0;
      s_slot = -1;
      s_stop = 0;
      if (R) {
        // offer the field to helpers right away (they start with the first
        // handshake): the record first, then a board entry
        sta(&R->team, (u64)t);
        __builtin_amdgcn_s_waitcnt(0);
        for (int b = 0; b < kBoard; ++b)
          if (atomicCAS(&board[b], 0u, (u32)f + 1u) == 0u) {
            s_slot = b;
            break;
          }
        atomicSub(B.queue + 1, 1ull);
      }
    }
    team_sync();
    for (u64 i = t0; i < (u64)nv; i += stride) {
      sa.s.g[i] = sa.s.gw[i] = i == (u64)B.field_src[f] ? 0ull : 0x7ff0000000000000ull;
      sa.s.fanth[i] = kAllOnes;
      sa.s.claim[i] = 0u;
    }
    for (u64 i = t0; i < (u64)nh; i += stride) {
      sa.s.as[i] = sa.s.asw[i] = Split{0x7ff0000000000000ull, kAllOnes};
    }
    // every wavefront's initial values are in the L2 before the field is
    // offered to helpers
    __builtin_amdgcn_s_waitcnt(0);
    team_sync();
    if (threadIdx.x < (u32)kWave) Ph::init_fan_(sa, B.field_src[f], &lctl);
    team_sync();
    if (threadIdx.x < (u32)kWave) Ph::begin(sa, 0);
    team_sync();
    const int slot = s_slot;
    bool global = false;  // counters in the gang record
    u64 count = 0;        // handshakes published
    int p = 0, ok = 1;
    for (;;) {
      if (threadIdx.x == 0) {
        const u64 done = ld(&sa.ctl->done);
        int nm = 1;
        if (slot >= 0) {
          sta(&R->prog, ld(&sa.ctl->tot[C_SEL]));
          nm = 1 + (int)min(ld(&R->join), (u64)(B.gang_max - 1));
          if (nm > 1 && !global) {
            // the first round with helpers: move the counters to the record
            const u64* src = (const u64*)&lctl;
            u64* dst = (u64*)&R->ctl;
            for (size_t w = 0; w < sizeof(Ctl) / sizeof(u64); ++w) dst[w] = src[w];
            sa.ctl = &R->ctl;
            global = true;
          }
          if (global && !done) {
            ++count;
            sta(&R->cnt[count & 1], 0ull);
            __builtin_amdgcn_s_waitcnt(0);
            sta(&R->word, (count << 8) | ((u64)p << 6) | (u64)nm);
          }
        }
        s_nm = nm;
        s_done = (int)done;
        s_word = count;
      }
      __syncthreads();
      if (s_done) break;
      if (!team_round<Ph, BS>(sa, p, 0, s_nm, R, (int)(s_word & 1), B.wait, &s_ok)) {
        ok = 0;
        break;
      }
      if (threadIdx.x < (u32)kWave) {
        Ph::begin(sa, 1 - p);
        if (threadIdx.x == 0 && (int64_t)ld(&sa.ctl->round) > B.max_rounds) sta(&sa.ctl->done, 1ull);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      p ^= 1;
    }
    if (slot >= 0 && threadIdx.x == 0) {
      // release the helpers, withdraw the offer, and wait until every helper
      // has left before the buffers take another field
      ++count;
      __builtin_amdgcn_s_waitcnt(0);
      sta(&R->word, (count << 8) | (1ull << 7));
      atomicExch(&board[slot], 0u);
      const u64 t_end = wall_clock64() + B.wait;
      while (ld(&R->left) < ld(&R->join)) {
        if (wall_clock64() > t_end) {
          s_stop = 1;  // a helper may still run: leave these buffers alone
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      l1_invalidate();
    }
    __syncthreads();
    const Ctl* c = sa.ctl;
    if (ok) {
      const int64_t off = B.field_off[f];
      for (u64 i = t0; i < (u64)nv; i += stride) B.out[off + i] = from_bits(lda(&sa.s.g[i]));
    }
    if (threadIdx.x == 0) {
      int64_t* st = B.fstat + (int64_t)f * kFieldStat;
      const u64 rounds = ld(&c->round);
      st[0] = field_status(ok, ld(&c->overflow) != 0, (int64_t)rounds > B.max_rounds, ld(&c->nonfinite) != 0,
                           ld(&c->badidx) != 0);
      st[1] = (int64_t)rounds;
      st[2] = (int64_t)ld(&c->tot[C_SEL]);
      st[3] = (int64_t)(ld(&c->tot[C_KIDS]) + ld(&c->tot[C_FANWIN]));
      st[4] = (int64_t)ld(&c->tot[C_FANS]);
      st[5] = (int64_t)ld(&c->peak);
      st[6] = (int64_t)ld(&c->tot[C_STALE]);
      st[7] = (int64_t)(wall_clock64() - t_start);
      st[8] = R ? (int64_t)ld(&R->join) : 0;
      st[9] = R ? (int64_t)ld(&R->hticks) : 0;
    }
    team_sync();
    if (s_stop) return;
  }
}

// Start of a batch launch: empty queue, fresh gang records and board, every
// field marked as not run (a kernel, not a memset, so that the launch can be
// captured in a graph and replayed).
// Geodesic Voronoi labels: per vertex the nearest of m fields (stored one
// after another, nv values each) and its index, ties to the lowest index.
__global__ void k_voronoi(const double* fields, int32_t m, int64_t nv, double* dist, int32_t* label) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
    double best = fields[v];
    int32_t arg = 0;
    for (int32_t i = 1; i < m; ++i) {
      const double d = fields[(int64_t)i * nv + v];
      if (d < best) {
        best = d;
        arg = i;
      }
    }
    dist[v] = best;
    label[v] = isfinite(best) ? arg : -1;
  }
}

__global__ void k_batch_reset(BatchDev B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    B.queue[0] = 0ull;
    B.queue[1] = 0ull;
  }
  if (i < B.n_fields) {
    GangRec* R = B.gang + i;
    R->word = 0ull;
    R->join = 0ull;
    R->left = 0ull;
    R->abort = 0ull;
    R->team = 0ull;
    R->prog = 0ull;
    R->hticks = 0ull;
    R->cnt[0] = R->cnt[1] = 0ull;
    B.fstat[(int64_t)i * kFieldStat] = kFieldNotRun;
  }
  if (i < kMaxXcc * kBoard) B.board[i] = 0u;
}

}  // namespace

// Work buffers of pch_geodesic_noalloc: one array per GPU, held until the
// process ends. Host code never uses this name as an address: each device's
// address comes from hipGetSymbolAddress (noalloc_scratch).
static __device__ __align__(256) char scratch[kScratchBytes];

int pch::set_error(int s, const std::string& msg) {
  t_err = msg;
  return s;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// The work buffers of one field: window pools, selection, hop queues, events,
// and the per-call tables (sources, cutoff table, predicted-distance table,
// round log). pch_geodesic keeps them in the mesh handle and grows them on
// demand; the no-alloc entry point carves them from its static scratch array.
struct WorkBufs {
  int64_t cap = 0, ecap = 0, acap = 0;
  Pool pool[2] = {};
  Pool sel = {};
  Pool hq[2] = {};
  Pool sorted = {};
  u32 *org_hist = nullptr, *org_ofs = nullptr;
  DistEv ev[2] = {};
  DistEv cand = {};
  AngEv aev = {};
  int32_t* dsrc = nullptr;
  double* dtable = nullptr;
  u32* dcdf = nullptr;  // [kCdfBins + 4]: histogram / cdf, the maximum, a pad word, the bin width
  int64_t* dlog = nullptr;
  int64_t dlog_cap = 0;
};

struct pch_mesh_s {
  pch::HostMesh host;
  int device = 0;
  // device copies
  HalfEdgeLine* hl = nullptr;
  double *phi = nullptr, *alpha = nullptr, *theta = nullptr;
  int32_t *twin = nullptr, *hv = nullptr, *coff = nullptr, *corner = nullptr;
  pch::Corner* crec = nullptr;
  uint8_t* flags = nullptr;
  // state (sized with the mesh)
  u64 *g = nullptr, *gw = nullptr, *fanth = nullptr;
  Split *as = nullptr, *asw = nullptr;
  u32* claim = nullptr;
  Ctl* ctl = nullptr;
  u32* hist = nullptr;
  // a captured graph of rounds_per_sync rounds, replayed while its launch
  // arguments stay the same
  hipGraphExec_t rg_exec = nullptr;
  hipStream_t rg_stream = nullptr;
  RoundArgs rg_args{};
  int rg_key[6] = {};
  // work buffers (grow on demand)
  WorkBufs w;
  int64_t hq_cap = 0, sorted_cap = 0, dsrc_cap = 0, dtable_cap = 0;
  std::vector<int64_t> last_log;
  int64_t last_rounds = 0;
};

namespace {

u64 bits_host(double x) {
  u64 u;
  std::memcpy(&u, &x, sizeof(u));
  return u;
}

template <class T>
hipError_t dalloc(T** p, int64_t n) {
  return hipMalloc((void**)p, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
}

void free_pool(Pool& P) {
  (void)hipFree(P.bb);
  (void)hipFree(P.pp);
  (void)hipFree(P.sk);
  (void)hipFree(P.es);
  P = Pool{};
}

hipError_t alloc_pool(Pool& P, int64_t n) {
  hipError_t e;
  if ((e = dalloc(&P.bb, n)) || (e = dalloc(&P.pp, n)) || (e = dalloc(&P.sk, n)) || (e = dalloc(&P.es, n)))
    return e;
  return hipSuccess;
}

void free_work(pch_mesh_s* M) {
  for (int i = 0; i < 2; ++i) {
    free_pool(M->w.pool[i]);
    (void)hipFree(M->w.ev[i].vq);
    (void)hipFree(M->w.ev[i].d);
    (void)hipFree(M->w.ev[i].xy);
    M->w.ev[i] = DistEv{};
  }
  (void)hipFree(M->w.cand.vq);
  (void)hipFree(M->w.cand.d);
  (void)hipFree(M->w.cand.xy);
  M->w.cand = DistEv{};
  free_pool(M->w.sel);
  free_pool(M->w.hq[0]);
  free_pool(M->w.hq[1]);
  M->hq_cap = 0;
  free_pool(M->w.sorted);
  M->sorted_cap = 0;
  (void)hipFree(M->w.aev.e);
  (void)hipFree(M->w.aev.D);
  (void)hipFree(M->w.aev.X);
  M->w.aev = AngEv{};
  M->w.cap = M->w.ecap = M->w.acap = 0;
}

pch_status ensure_work(pch_mesh_s* M, int64_t cap, bool hop_queues) {
  if (cap <= M->w.cap && (!hop_queues || M->hq_cap >= M->w.cap)) return PCH_OK;
  if (cap <= M->w.cap) {
    // the hop queues are allocated on first use
    HIP_TRY(alloc_pool(M->w.hq[0], M->w.cap));
    HIP_TRY(alloc_pool(M->w.hq[1], M->w.cap));
    M->hq_cap = M->w.cap;
    return PCH_OK;
  }
  free_work(M);
  const int64_t ecap = 4 * cap, acap = cap;
  for (int i = 0; i < 2; ++i) {
    HIP_TRY(alloc_pool(M->w.pool[i], cap));
    HIP_TRY(dalloc(&M->w.ev[i].vq, ecap));
    HIP_TRY(dalloc(&M->w.ev[i].d, ecap));
    HIP_TRY(dalloc(&M->w.ev[i].xy, ecap));
  }
  HIP_TRY(dalloc(&M->w.cand.vq, ecap));
  HIP_TRY(dalloc(&M->w.cand.d, ecap));
  HIP_TRY(dalloc(&M->w.cand.xy, ecap));
  HIP_TRY(alloc_pool(M->w.sel, cap));
  if (hop_queues) {
    HIP_TRY(alloc_pool(M->w.hq[0], cap));
    HIP_TRY(alloc_pool(M->w.hq[1], cap));
    M->hq_cap = cap;
  }
  HIP_TRY(dalloc(&M->w.aev.e, acap));
  HIP_TRY(dalloc(&M->w.aev.D, acap));
  HIP_TRY(dalloc(&M->w.aev.X, acap));
  M->w.cap = cap;
  M->w.ecap = ecap;
  M->w.acap = acap;
  return PCH_OK;
}

// Device memory that the no-alloc entry point takes its work buffers from.
struct ScratchArena {
  char* base;
  size_t bytes;
};

// Lays out the work buffers of one field with pool capacity cap (and the
// same event capacities as pch_geodesic) from base, each array 256-byte
// aligned; returns the bytes they take. Assigns w only when they fit in avail.
// The sources, cutoff table and predicted-distance table come first, so a
// larger cap leaves them where they are.
size_t carve_work(WorkBufs& w, char* base, size_t avail, int64_t cap, int64_t nsrc, int64_t ntable, bool cdf) {
  const int64_t ecap = 4 * cap, acap = cap;
  size_t at = 0;
  auto take = [&](size_t n) {
    const size_t o = at;
    at += (n + 255) & ~(size_t)255;
    return o;
  };
  const size_t o_src = take(sizeof(int32_t) * (size_t)kNoallocMaxSources);
  const size_t o_tab = ntable > 0 ? take(sizeof(double) * ntable) : 0;
  const size_t o_cdf = cdf ? take(sizeof(u32) * (kCdfBins + 4)) : 0;
  (void)nsrc;
  size_t o_pool[3][4], o_ev[3][3], o_ae[3];
  for (auto& q : o_pool) {
    q[0] = take(sizeof(double2) * cap);
    q[1] = take(sizeof(double2) * cap);
    q[2] = take(sizeof(double2) * cap);
    q[3] = take(sizeof(int2) * cap);
  }
  for (auto& q : o_ev) {
    q[0] = take(sizeof(int2) * ecap);
    q[1] = take(sizeof(double) * ecap);
    q[2] = take(sizeof(double2) * ecap);
  }
  o_ae[0] = take(sizeof(int32_t) * acap);
  o_ae[1] = take(sizeof(double) * acap);
  o_ae[2] = take(sizeof(double) * acap);
  if (at > avail) return at;
  auto pool_at = [&](const size_t* q) {
    return Pool{reinterpret_cast<double2*>(base + q[0]), reinterpret_cast<double2*>(base + q[1]),
                reinterpret_cast<double2*>(base + q[2]), reinterpret_cast<int2*>(base + q[3])};
  };
  auto ev_at = [&](const size_t* q) {
    return DistEv{reinterpret_cast<int2*>(base + q[0]), reinterpret_cast<double*>(base + q[1]),
                  reinterpret_cast<double2*>(base + q[2])};
  };
  w = WorkBufs{};
  w.cap = cap;
  w.ecap = ecap;
  w.acap = acap;
  w.pool[0] = pool_at(o_pool[0]);
  w.pool[1] = pool_at(o_pool[1]);
  w.sel = pool_at(o_pool[2]);
  w.ev[0] = ev_at(o_ev[0]);
  w.ev[1] = ev_at(o_ev[1]);
  w.cand = ev_at(o_ev[2]);
  w.aev = AngEv{reinterpret_cast<int32_t*>(base + o_ae[0]), reinterpret_cast<double*>(base + o_ae[1]),
                reinterpret_cast<double*>(base + o_ae[2])};
  w.dsrc = reinterpret_cast<int32_t*>(base + o_src);
  w.dtable = ntable > 0 ? reinterpret_cast<double*>(base + o_tab) : nullptr;
  w.dcdf = cdf ? reinterpret_cast<u32*>(base + o_cdf) : nullptr;
  return at;
}

pch_status upload_mesh(pch_mesh_s* M, hipStream_t st) {
  const pch::HostMesh& H = M->host;
  // distance events name their half-edge as 4 e + k in 32 bits
  if (H.nh >= ((int64_t)1 << 29)) return set_err(PCH_EINVAL, "mesh too large: at most 2^29 - 1 half-edges");
  HIP_TRY(dalloc(&M->hl, H.nh));
  HIP_TRY(dalloc(&M->phi, H.nh));
  HIP_TRY(dalloc(&M->alpha, H.nh));
  HIP_TRY(dalloc(&M->twin, H.nh));
  HIP_TRY(dalloc(&M->hv, H.nh));
  HIP_TRY(dalloc(&M->corner, H.nh));
  HIP_TRY(dalloc(&M->crec, H.nh));
  HIP_TRY(dalloc(&M->theta, H.nv));
  HIP_TRY(dalloc(&M->flags, H.nv));
  HIP_TRY(dalloc(&M->coff, H.nv + 1));
  HIP_TRY(dalloc(&M->g, H.nv));
  HIP_TRY(dalloc(&M->as, H.nh));
  HIP_TRY(dalloc(&M->gw, H.nv));
  HIP_TRY(dalloc(&M->asw, H.nh));
  HIP_TRY(dalloc(&M->fanth, H.nv));
  HIP_TRY(dalloc(&M->claim, H.nv));
  HIP_TRY(dalloc(&M->ctl, 1));
  HIP_TRY(dalloc(&M->hist, kHistBins));
  {
    std::vector<HalfEdgeLine> lines((size_t)H.nh);
    for (int64_t j = 0; j < H.nh; ++j) lines[j] = HalfEdgeLine{H.he[j], H.hang[j]};
    HIP_TRY(hipMemcpyAsync(M->hl, lines.data(), sizeof(HalfEdgeLine) * H.nh, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));  // before the staging vector goes away
  }
  HIP_TRY(hipMemcpyAsync(M->phi, H.phi.data(), sizeof(double) * H.nh, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(M->alpha, H.alpha.data(), sizeof(double) * H.nh, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(M->twin, H.twin.data(), sizeof(int32_t) * H.nh, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(M->hv, H.hv.data(), sizeof(int32_t) * H.nh, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(M->corner, H.corner.data(), sizeof(int32_t) * H.nh, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(M->crec, H.crec.data(), sizeof(pch::Corner) * H.nh, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(M->theta, H.theta.data(), sizeof(double) * H.nv, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(M->flags, H.flags.data(), H.nv, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(M->coff, H.coff.data(), sizeof(int32_t) * (H.nv + 1), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(M->hist, 0, sizeof(u32) * kHistBins, st));
  HIP_TRY(hipStreamSynchronize(st));
  return PCH_OK;
}

void free_mesh(pch_mesh_s* M) {
  if (M->rg_exec) (void)hipGraphExecDestroy(M->rg_exec);
  if (M->rg_stream) (void)hipStreamDestroy(M->rg_stream);
  free_work(M);
  (void)hipFree(M->hl);
  (void)hipFree(M->phi);
  (void)hipFree(M->alpha);
  (void)hipFree(M->twin);
  (void)hipFree(M->hv);
  (void)hipFree(M->corner);
  (void)hipFree(M->crec);
  (void)hipFree(M->theta);
  (void)hipFree(M->flags);
  (void)hipFree(M->coff);
  (void)hipFree(M->g);
  (void)hipFree(M->as);
  (void)hipFree(M->gw);
  (void)hipFree(M->asw);
  (void)hipFree(M->fanth);
  (void)hipFree(M->claim);
  (void)hipFree(M->ctl);
  (void)hipFree(M->hist);
  (void)hipFree(M->w.dsrc);
  (void)hipFree(M->w.dtable);
  (void)hipFree(M->w.dcdf);
  (void)hipFree(M->w.dlog);
  (void)hipFree(M->w.org_hist);
  (void)hipFree(M->w.org_ofs);
}

pch_status finish_create(pch_mesh_s* M, void* stream, pch_mesh* out) {
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipGetDevice(&M->device));
  pch_status s = upload_mesh(M, st);
  if (s != PCH_OK) {
    free_mesh(M);
    delete M;
    return s;
  }
  *out = M;
  return PCH_OK;
}

RoundArgs make_args(pch_mesh_s* M, const WorkBufs& w, const pch_options& o) {
  RoundArgs a{};  // zeroed padding: captured round graphs compare arguments bytewise
  a.m = DevMesh{M->hl,    M->phi,    M->alpha, M->twin, M->hv, M->theta, M->flags, M->coff,
                 M->corner, M->crec, (int32_t)M->host.nv, (int32_t)M->host.nh};
  a.s = DevState{M->g, M->as, M->fanth, M->claim, M->gw, M->asw};
  a.pool[0] = w.pool[0];
  a.pool[1] = w.pool[1];
  a.sel = w.sel;
  a.hq[0] = w.hq[0];
  a.hq[1] = w.hq[1];
  a.hops = o.hops;
  a.org_shift = -1;
  if (o.organize) {
    int bitlen = 0;
    while (((M->host.nh - 1) >> bitlen) > 0) ++bitlen;
    a.org_shift = bitlen > 12 ? bitlen - 12 : 0;  // (nh - 1) >> org_shift < kOrgBuckets
  }
  a.sorted = w.sorted;
  a.org_hist = w.org_hist;
  a.org_ofs = w.org_ofs;
  a.ev[0] = w.ev[0];
  a.ev[1] = w.ev[1];
  a.cand = w.cand;
  a.aev = w.aev;
  a.ctl = M->ctl;
  a.hist = M->hist;
  a.log = o.collect_stats ? w.dlog : nullptr;
  a.max_log = o.collect_stats ? w.dlog_cap : 0;
  a.cap = w.cap;
  a.ecap = w.ecap;
  a.acap = w.acap;
  a.k = o.k;
  a.mode = o.select_mode;
  a.eps = o.eps_tiny;
  a.ch_on = (o.filters & 1) != 0;
  a.ich_on = (o.filters & 2) != 0;
  a.full_fan = (o.filters & 4) != 0;
  a.retest = (o.filters & 8) != 0;
  a.table = (o.select_mode == PCH_SELECT_TABLE) ? w.dtable : nullptr;
  a.n_table = (o.select_mode == PCH_SELECT_TABLE) ? o.n_cutoff : 0;
  a.cdf = w.dcdf;
  a.pbin = 0.0;
  a.w0 = o.w0 > 0.0 ? o.w0 : 4.0;
  a.counts = (o.counts != 0 || o.collect_stats != 0) ? 1 : 0;
  return a;
}

constexpr int kRoundEvents = 5;  // timing events of one timed round

int grid_for(int64_t work, int max_blocks) {
  int64_t b = (work + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

// Enqueue one round with input parity p (its set-up already ran: the initial
// k_begin or the previous round's k_events3). ev0/ev1 (optional) bracket the
// propagation launches: one for all hops when fused, else one per hop.
// Grids: the pool scan uses pool_blocks; propagation is sized for about twice
// k windows; event passes and histograms use few blocks because their work is
// small and the last-block ticket serializes one atomic per block.
// One fused propagation launch with the hop lists that a.hops needs.
void launch_fused(const RoundArgs& a, int p, hipStream_t st, int blocks) {
  switch (a.hops <= 2 ? 1 : a.hops - 1) {
    case 1: k_propagate_fused<1><<<blocks, kBlock, 0, st>>>(a, p); break;
    case 2: k_propagate_fused<2><<<blocks, kBlock, 0, st>>>(a, p); break;
    case 3: k_propagate_fused<3><<<blocks, kBlock, 0, st>>>(a, p); break;
    case 4: k_propagate_fused<4><<<blocks, kBlock, 0, st>>>(a, p); break;
    default: k_propagate_fused<5><<<blocks, kBlock, 0, st>>>(a, p); break;
  }
}

// Workgroups of the fused scan-and-propagation kernel for `hops` that the
// current device holds at once (occupancy times compute units), per device.
int resident_blocks(int hops, bool reg) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  const int nl = hops <= 2 ? 1 : (hops - 1 > 5 ? 5 : hops - 1);
  const auto key = std::make_tuple(dev, nl, reg ? 1 : 0);
  std::lock_guard<std::mutex> lock(mu);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const void* fn = nullptr;
  if (reg) {
    const void* r[5] = {(const void*)k_select_propagate_r<1>, (const void*)k_select_propagate_r<2>,
                        (const void*)k_select_propagate_r<3>, (const void*)k_select_propagate_r<4>,
                        (const void*)k_select_propagate_r<5>};
    fn = r[nl - 1];
  } else {
    const void* f[5] = {(const void*)k_select_propagate<1>, (const void*)k_select_propagate<2>,
                        (const void*)k_select_propagate<3>, (const void*)k_select_propagate<4>,
                        (const void*)k_select_propagate<5>};
    fn = f[nl - 1];
  }
  int per_cu = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 256;
  const int n = per_cu * ncu;
  cache[key] = n;
  return n;
}

// The pool scan and the propagation of all hops in one launch (reg: the
// lists hold only the second hopping child of a window).
void launch_select_fused(const RoundArgs& a, int p, hipStream_t st, int blocks, bool reg) {
  if (reg) {
    switch (a.hops <= 2 ? 1 : a.hops - 1) {
      case 1: k_select_propagate_r<1><<<blocks, kBlock, 0, st>>>(a, p); break;
      case 2: k_select_propagate_r<2><<<blocks, kBlock, 0, st>>>(a, p); break;
      case 3: k_select_propagate_r<3><<<blocks, kBlock, 0, st>>>(a, p); break;
      case 4: k_select_propagate_r<4><<<blocks, kBlock, 0, st>>>(a, p); break;
      default: k_select_propagate_r<5><<<blocks, kBlock, 0, st>>>(a, p); break;
    }
    return;
  }
  switch (a.hops <= 2 ? 1 : a.hops - 1) {
    case 1: k_select_propagate<1><<<blocks, kBlock, 0, st>>>(a, p); break;
    case 2: k_select_propagate<2><<<blocks, kBlock, 0, st>>>(a, p); break;
    case 3: k_select_propagate<3><<<blocks, kBlock, 0, st>>>(a, p); break;
    case 4: k_select_propagate<4><<<blocks, kBlock, 0, st>>>(a, p); break;
    default: k_select_propagate<5><<<blocks, kBlock, 0, st>>>(a, p); break;
  }
}

// Round launch plan: kSplit = partition, then propagation (fused hops or one
// launch per hop); kScanFused = the pool scan inside the fused propagation;
// kScanFusedReg = the same with the first hopping child of each window kept
// in registers.
enum RoundPlan { kSplit = 0, kScanFused = 1, kScanFusedReg = 2 };

void enqueue_round(const RoundArgs& a, int p, hipStream_t st, int pool_blocks, int prop_blocks, bool kth, bool fused,
                   const hipEvent_t* ev = nullptr, RoundPlan plan = kSplit) {
  // ev (optional): kRoundEvents events bracketing the phases: selection,
  // organization, propagation, events
  if (ev) (void)hipEventRecord(ev[0], st);
  if (kth)
    for (int pass = 0; pass < 3; ++pass) k_hist<<<kSmallGrid, kBlock, 0, st>>>(a, p, pass);
  if (plan == kScanFused || plan == kScanFusedReg) {
    if (ev) (void)hipEventRecord(ev[1], st);
    if (ev) (void)hipEventRecord(ev[2], st);
    launch_select_fused(a, p, st, pool_blocks, plan == kScanFusedReg);
    if (ev) (void)hipEventRecord(ev[3], st);
    k_events2<<<kSmallGrid, kBlock, 0, st>>>(a, p);
    k_events3<<<kSmallGrid, kBlock, 0, st>>>(a, p);
    if (ev) (void)hipEventRecord(ev[4], st);
    return;
  }
  k_partition<<<pool_blocks, kBlock, 0, st>>>(a, p);
  if (ev) (void)hipEventRecord(ev[1], st);
  if (a.org_shift >= 0) {
    k_org_scan<<<1, 1024, 0, st>>>(a);
    k_org_scatter<<<prop_blocks, kBlock, 0, st>>>(a);
  }
  if (ev) (void)hipEventRecord(ev[2], st);
  if (fused)
    launch_fused(a, p, st, prop_blocks);
  else
    for (int h = 1; h <= a.hops; ++h) k_propagate<<<prop_blocks, kBlock, 0, st>>>(a, p, h);
  if (ev) (void)hipEventRecord(ev[3], st);
  k_events2<<<kSmallGrid, kBlock, 0, st>>>(a, p);
  k_events3<<<kSmallGrid, kBlock, 0, st>>>(a, p);
  if (ev) (void)hipEventRecord(ev[4], st);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* pch_last_error(void) { return t_err.c_str(); }

const char* pch_field_status_string(int64_t s) {
  switch (s) {
    case PCH_FIELD_OK: return "ok";
    case PCH_FIELD_OVERFLOW: return "pool overflow (rerun)";
    case PCH_FIELD_MAX_ROUNDS: return "round limit (rerun)";
    case PCH_FIELD_ABANDONED: return "gang stopped waiting (rerun)";
    case PCH_FIELD_NOT_RUN: return "not finished (rerun)";
    case PCH_FIELD_NONFINITE: return "non-finite window geometry";
    case PCH_FIELD_BAD_INDEX: return "index outside the mesh";
  }
  return "unknown field status";
}

const char* pch_status_string(pch_status s) {
  switch (s) {
    case PCH_OK: return "ok";
    case PCH_EINVAL: return "invalid argument";
    case PCH_EMESH: return "invalid mesh";
    case PCH_ENOMEM: return "out of memory";
    case PCH_EDEVICE: return "device error";
    case PCH_EOVERFLOW: return "window pool limit exceeded";
    case PCH_ENUMERIC: return "non-finite window geometry";
  }
  return "unknown status";
}

void pch_options_default(pch_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->select_mode = PCH_SELECT_KTH;
  o->filters = 3;
  o->k = 16384;
  o->eps_tiny = 0.0;
  o->pool_capacity = 0;
  o->pool_limit = 0;
  o->collect_stats = 0;
  o->rounds_per_sync = 16;
  o->cutoff_table = nullptr;
  o->n_cutoff = 0;
  o->hops = 1;
  o->counts = 1;
  o->fuse_hops = 1;
  o->fuse_scan = 2;
  o->round_graph = 0;
}

pch_status pch_mesh_create_from_lengths(const int32_t* faces, int64_t nf, int64_t nv, const double* he_len,
                                        void* hip_stream, pch_mesh* out) {
  if (!faces || !he_len || !out) return set_err(PCH_EINVAL, "null pointer argument");
  *out = nullptr;
  pch_mesh_s* M = new (std::nothrow) pch_mesh_s();
  if (!M) return set_err(PCH_ENOMEM, "host allocation failed");
  std::string msg;
  int rc = pch::build_host_mesh(faces, nf, nv, he_len, M->host, msg);
  if (rc != PCH_OK) {
    delete M;
    return set_err((pch_status)rc, msg);
  }
  return finish_create(M, hip_stream, out);
}

pch_status pch_mesh_create(const double* xyz, int64_t nv, const int32_t* faces, int64_t nf, void* hip_stream,
                           pch_mesh* out) {
  if (!xyz || !faces || !out) return set_err(PCH_EINVAL, "null pointer argument");
  if (nv < 1 || nf < 1) return set_err(PCH_EINVAL, "mesh needs at least one face and one vertex");
  std::vector<double> len;
  std::string msg;
  int rc = pch::lengths_from_xyz(xyz, nv, faces, nf, len, msg);
  if (rc != PCH_OK) return set_err((pch_status)rc, msg);
  return pch_mesh_create_from_lengths(faces, nf, nv, len.data(), hip_stream, out);
}

void pch_mesh_destroy(pch_mesh M) {
  if (!M) return;
  free_mesh(M);
  delete M;
}

pch_status pch_mesh_info(pch_mesh M, int64_t* nv, int64_t* nf, int64_t* nbhe, int64_t* npseudo) {
  if (!M) return set_err(PCH_EINVAL, "null mesh");
  if (nv) *nv = M->host.nv;
  if (nf) *nf = M->host.nf;
  if (nbhe) *nbhe = M->host.n_boundary_he;
  if (npseudo) *npseudo = M->host.n_pseudo;
  return PCH_OK;
}

pch_status pch_mesh_vertex_tables(pch_mesh M, double* theta, uint8_t* flags) {
  if (!M) return set_err(PCH_EINVAL, "null mesh");
  if (theta) std::memcpy(theta, M->host.theta.data(), sizeof(double) * M->host.nv);
  if (flags) std::memcpy(flags, M->host.flags.data(), M->host.nv);
  return PCH_OK;
}

pch_status pch_round_log(pch_mesh M, int64_t* out, int64_t max_rounds, int64_t* n_rounds) {
  if (!M) return set_err(PCH_EINVAL, "null mesh");
  if (n_rounds) *n_rounds = M->last_rounds;
  if (out && max_rounds > 0) {
    const int64_t n = std::min<int64_t>(max_rounds, (int64_t)M->last_log.size() / C_NUM);
    std::memcpy(out, M->last_log.data(), sizeof(int64_t) * C_NUM * n);
  }
  return PCH_OK;
}

// Algorithm 1 on one mesh. sc == nullptr: the work buffers live in the mesh
// handle and grow on demand (pch_geodesic); otherwise they are carved from
// the arena and nothing is allocated (pch_geodesic_noalloc).
static pch_status geodesic_core(pch_mesh M, const int32_t* sources, int32_t m, double* dist, void* hip_stream,
                                const pch_options* opts, pch_stats* stats, const ScratchArena* sc) {
  auto t_start = std::chrono::steady_clock::now();
  if (!M || !sources || !dist) return set_err(PCH_EINVAL, "null pointer argument");
  if (m < 1) return set_err(PCH_EINVAL, "need at least one source vertex");
  pch_options o;
  pch_options_default(&o);
  if (opts) o = *opts;
  if (o.select_mode != PCH_SELECT_KTH && o.select_mode != PCH_SELECT_DELTA && o.select_mode != PCH_SELECT_TABLE &&
      o.select_mode != PCH_SELECT_LEARNED && o.select_mode != PCH_SELECT_STRIDED)
    return set_err(PCH_EINVAL, "unknown select_mode");
  if (o.select_mode == PCH_SELECT_LEARNED && !o.predicted)
    return set_err(PCH_EINVAL, "learned selection needs predicted distances");
  if (!(o.delta0 >= 0.0)) return set_err(PCH_EINVAL, "delta0 must be >= 0");
  if (o.collect_timing < 0) return set_err(PCH_EINVAL, "collect_timing must be >= 0");
  if (o.k < 1) return set_err(PCH_EINVAL, "k must be >= 1");
  if (o.select_mode == PCH_SELECT_TABLE && (o.n_cutoff < 0 || (o.n_cutoff > 0 && !o.cutoff_table)))
    return set_err(PCH_EINVAL, "cutoff table missing");
  if (!(o.eps_tiny >= 0.0)) return set_err(PCH_EINVAL, "eps_tiny must be >= 0");
  if (o.rounds_per_sync < 1) o.rounds_per_sync = 16;
  if (o.hops == 0) o.hops = 1;
  if (o.hops < 1 || o.hops > kMaxHops) return set_err(PCH_EINVAL, "hops must be in [1, 16]");
  const bool fused_hops = o.fuse_hops != 0 && o.hops <= kFuseHops;
  if (sc) {
    if (m > kNoallocMaxSources) return set_err(PCH_EINVAL, "the no-alloc entry point takes at most 1024 sources");
    if (o.collect_timing || o.collect_stats || o.organize || (o.hops > 1 && !fused_hops))
      return set_err(PCH_EINVAL,
                     "the no-alloc entry point does not take collect_timing, collect_stats, organize or unfused hops");
  }
  const pch::HostMesh& H = M->host;
  // the sources, sorted and without duplicates (a stack array for up to
  // kNoallocMaxSources of them)
  int32_t src_small[kNoallocMaxSources];
  std::vector<int32_t> src_big;
  int32_t* src = src_small;
  if (m > kNoallocMaxSources) {
    src_big.assign(sources, sources + m);
    src = src_big.data();
  } else {
    std::memcpy(src_small, sources, sizeof(int32_t) * (size_t)m);
  }
  for (int32_t i = 0; i < m; ++i)
    if (src[i] < 0 || src[i] >= H.nv) return set_err(PCH_EINVAL, "source vertex out of range");
  std::sort(src, src + m);
  const int nsrc = (int)(std::unique(src, src + m) - src);
  hipStream_t st = (hipStream_t)hip_stream;
  int cur_dev = 0;
  HIP_TRY(hipGetDevice(&cur_dev));
  if (cur_dev != M->device) return set_err(PCH_EINVAL, "mesh was created on another device");
  const bool use_table = o.select_mode == PCH_SELECT_TABLE && o.n_cutoff > 0;
  int64_t cap = o.pool_capacity > 0 ? o.pool_capacity : std::max<int64_t>(1 << 18, 2 * H.nh);
  if (o.pool_limit > 0 && cap > o.pool_limit) cap = o.pool_limit;
  // the work buffers: the mesh's own, or carved from the arena
  WorkBufs wl;
  WorkBufs& w = sc ? wl : M->w;
  if (sc) {
    const size_t need = carve_work(wl, sc->base, sc->bytes, cap, nsrc, use_table ? o.n_cutoff : 0,
                                   o.select_mode == PCH_SELECT_LEARNED);
    if (need > sc->bytes)
      return set_err(PCH_EOVERFLOW, "the field needs " + std::to_string(need >> 20) +
                                        " MiB of work buffers, more than the no-alloc scratch of " +
                                        std::to_string(sc->bytes >> 20) + " MiB");
  } else if ((int64_t)nsrc > M->dsrc_cap) {
    (void)hipFree(M->w.dsrc);
    M->w.dsrc = nullptr;
    HIP_TRY(dalloc(&M->w.dsrc, (int64_t)nsrc));
    M->dsrc_cap = (int64_t)nsrc;
  }
  HIP_TRY(hipMemcpyAsync(w.dsrc, src, sizeof(int32_t) * (size_t)nsrc, hipMemcpyHostToDevice, st));
  if (use_table) {
    if (!sc && o.n_cutoff > M->dtable_cap) {
      (void)hipFree(M->w.dtable);
      M->w.dtable = nullptr;
      HIP_TRY(dalloc(&M->w.dtable, o.n_cutoff));
      M->dtable_cap = o.n_cutoff;
    }
    HIP_TRY(hipMemcpyAsync(w.dtable, o.cutoff_table, sizeof(double) * o.n_cutoff, hipMemcpyHostToDevice, st));
  }
  double delta0 = o.delta0;
  if (delta0 == 0.0) {
    double sum = 0.0;
    for (int64_t j = 0; j < H.nh; ++j) sum += H.he[j].L;
    delta0 = 2.0 * (sum / (double)H.nh);
  }
  double pbin = 0.0;
  if (o.select_mode == PCH_SELECT_LEARNED) {
    // the table (kCdfBins + 1 words), a pad word, then the bin width (8-byte aligned)
    if (!w.dcdf) HIP_TRY(dalloc(&M->w.dcdf, kCdfBins + 4));
    double* dpbin = reinterpret_cast<double*>(w.dcdf + kCdfBins + 2);
    enqueue_pred_cdf(PredFields{o.predicted, nullptr, nullptr, H.nv, 1, w.dcdf, dpbin}, st);
    HIP_TRY(hipMemcpyAsync(&pbin, dpbin, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (!(pbin > 0.0)) return set_err(PCH_EINVAL, "predicted distances must be positive");
  }
  const int64_t log_rounds = 1 << 18;
  if (o.collect_stats && M->w.dlog_cap < log_rounds) {
    (void)hipFree(M->w.dlog);
    M->w.dlog = nullptr;
    HIP_TRY(dalloc(&M->w.dlog, log_rounds * C_NUM));
    M->w.dlog_cap = log_rounds;
  }
  int64_t restarts = 0;
  Ctl host_ctl, ctl_init;
  // optional per-launch timing of the propagation kernel
  std::vector<hipEvent_t> tev;
  if (o.collect_timing) {  // never with the arena (rejected above)
    tev.resize(kRoundEvents * (size_t)o.rounds_per_sync);
    for (auto& e : tev) HIP_TRY(hipEventCreate(&e));
  }
  struct EvGuard {
    std::vector<hipEvent_t>& v;
    ~EvGuard() {
      for (auto e : v) (void)hipEventDestroy(e);
    }
  } ev_guard{tev};
  int64_t prop_n = 0, timed_rounds = 0;
  double phase_ms[4] = {0.0, 0.0, 0.0, 0.0};
  RoundPlan plan_used = kSplit;
  int fused_wg = 0;
  for (;;) {
    // the hop queues in device memory serve only one launch per hop (fused
    // hops keep their windows in LDS)
    if (sc) {
      // a restart with a larger pool stays inside the arena or fails
      const size_t need = carve_work(wl, sc->base, sc->bytes, cap, nsrc, use_table ? o.n_cutoff : 0,
                                     o.select_mode == PCH_SELECT_LEARNED);
      if (need > sc->bytes) return set_err(PCH_EOVERFLOW, "window pool outgrew the no-alloc scratch");
    } else {
      pch_status s = ensure_work(M, cap, o.hops > 1 && !fused_hops);
      if (s != PCH_OK) return s;
    }
    if (!sc && o.organize && M->sorted_cap < M->w.cap) {
      free_pool(M->w.sorted);
      HIP_TRY(alloc_pool(M->w.sorted, M->w.cap));
      M->sorted_cap = M->w.cap;
      if (!M->w.org_hist) {
        HIP_TRY(dalloc(&M->w.org_hist, kOrgBuckets));
        HIP_TRY(dalloc(&M->w.org_ofs, kOrgBuckets));
        HIP_TRY(hipMemsetAsync(M->w.org_hist, 0, sizeof(u32) * kOrgBuckets, st));
      }
    }
    RoundArgs a = make_args(M, w, o);
    a.pbin = pbin;
    const int fill_blocks = 1024;
    k_fill_u64<<<fill_blocks, kBlock, 0, st>>>(M->g, H.nv, bits_host(INFINITY));
    k_fill_u64<<<fill_blocks, kBlock, 0, st>>>(M->gw, H.nv, bits_host(INFINITY));
    k_fill_split<<<fill_blocks, kBlock, 0, st>>>(M->as, H.nh, bits_host(INFINITY), kAllOnes);
    k_fill_split<<<fill_blocks, kBlock, 0, st>>>(M->asw, H.nh, bits_host(INFINITY), kAllOnes);
    k_fill_u64<<<fill_blocks, kBlock, 0, st>>>(M->fanth, H.nv, kAllOnes);
    k_fill_u32<<<fill_blocks, kBlock, 0, st>>>(M->claim, H.nv, 0u);
    std::memset(&ctl_init, 0, sizeof(ctl_init));
    ctl_init.kmin[0] = ctl_init.kmin[1] = kAllOnes;
    ctl_init.delta = delta0;
    ctl_init.lfac = 1.0;
    HIP_TRY(hipMemcpyAsync(M->ctl, &ctl_init, sizeof(Ctl), hipMemcpyHostToDevice, st));
    k_set_sources<<<(nsrc + kBlock - 1) / kBlock, kBlock, 0, st>>>(M->g, M->gw, w.dsrc, nsrc);
    k_init_fans<<<(nsrc + kBlock - 1) / kBlock, kBlock, 0, st>>>(a, w.dsrc, nsrc);
    k_begin<<<1, kWave, 0, st>>>(a, 0);
    HIP_TRY(hipGetLastError());
    // the pool scan is sized from the largest pool seen so far (twice it, at
    // least 2k windows); its grid-stride loop covers any larger pool
    int pool_blocks = grid_for(std::max<int64_t>(2 * o.k, (int64_t)1 << 16), 1024);
    const int prop_blocks = grid_for(std::max<int64_t>(2 * o.k, 1), 2048);
    const bool fused = fused_hops;
    // the histogram passes serve the k-th-key rule (and a cutoff table's
    // rounds after the table); the other rules set their cutoff in the set-up
    const bool kth = o.select_mode == PCH_SELECT_KTH || o.select_mode == PCH_SELECT_TABLE;
    // the strided selection runs the pool scan on k threads (whole
    // workgroups): each selects the nearest of its windows
    const bool strided = o.select_mode == PCH_SELECT_STRIDED;
    if (strided) pool_blocks = grid_for(o.k, 1 << 30);
    // the pool scan runs inside the fused propagation unless the round needs
    // the whole selection first (strided selection, grouping by edge)
    const RoundPlan plan = (fused && o.fuse_scan != 0 && !strided && !o.organize)
                               ? (o.fuse_scan == 2 ? kScanFusedReg : kScanFused)
                               : kSplit;
    plan_used = plan;
    // the fused scan runs on as many workgroups as the device holds at once:
    // none starts after others have finished, and the tickets balance the
    // rest (scan_ticket)
    const int fused_blocks = plan == kSplit ? 0 : resident_blocks(a.hops, plan == kScanFusedReg);
    if (fused_blocks > 0) pool_blocks = fused_blocks;
    fused_wg = fused_blocks;
    int p = 0;
    bool overflow = false;
    for (double& x : phase_ms) x = 0.0;
    prop_n = 0;
    timed_rounds = 0;
    u64 rounds_before = 0;
    // rounds_per_sync rounds from a captured graph: only without timing
    // events, with an even chunk (every chunk starts at parity 0), and not in
    // the no-alloc entry point (instantiating a graph allocates)
    const bool graph = o.round_graph != 0 && !o.collect_timing && o.rounds_per_sync % 2 == 0 && !sc;
    // Rounds enqueued before the next poll of the control block: all
    // rounds_per_sync while the pool grows; while it shrinks, about the
    // rounds it has left at its current rate (at least 2), so that few empty
    // rounds are enqueued after the last one.
    int chunk = o.rounds_per_sync;
    u64 n_prev = 0;
    for (;;) {
      if (graph && chunk == o.rounds_per_sync && p == 0) {
        const int key[6] = {pool_blocks, prop_blocks, kth ? 1 : 0, fused ? 1 : 0, (int)plan, o.rounds_per_sync};
        if (!M->rg_exec || std::memcmp(key, M->rg_key, sizeof key) != 0 ||
            std::memcmp(&a, &M->rg_args, sizeof a) != 0) {
          if (M->rg_exec) (void)hipGraphExecDestroy(M->rg_exec);
          M->rg_exec = nullptr;
          if (!M->rg_stream) HIP_TRY(hipStreamCreateWithFlags(&M->rg_stream, hipStreamNonBlocking));
          hipGraph_t gr;
          HIP_TRY(hipStreamBeginCapture(M->rg_stream, hipStreamCaptureModeThreadLocal));
          for (int r = 0; r < o.rounds_per_sync; ++r)
            enqueue_round(a, r & 1, M->rg_stream, pool_blocks, prop_blocks, kth, fused, nullptr, plan);
          HIP_TRY(hipStreamEndCapture(M->rg_stream, &gr));
          const hipError_t e = hipGraphInstantiate(&M->rg_exec, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          if (e != hipSuccess) {
            M->rg_exec = nullptr;
            return set_err(PCH_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
          }
          std::memcpy(M->rg_key, key, sizeof key);
          std::memcpy(&M->rg_args, &a, sizeof a);
        }
        HIP_TRY(hipGraphLaunch(M->rg_exec, st));
      } else {
        for (int r = 0; r < chunk; ++r) {
          const bool timed = o.collect_timing && ((rounds_before + (u64)r) % (u64)o.collect_timing == 0);
          enqueue_round(a, p, st, pool_blocks, prop_blocks, kth, fused,
                        timed ? &tev[kRoundEvents * (size_t)r] : nullptr, plan);
          p ^= 1;
        }
      }
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(&host_ctl, M->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (o.collect_timing) {
        const u64 ran = host_ctl.round - rounds_before;
        for (u64 r = 0; r < ran && r < (u64)chunk; ++r) {
          if ((rounds_before + r) % (u64)o.collect_timing != 0) continue;
          const hipEvent_t* ev = &tev[kRoundEvents * (size_t)r];
          // phases in pch_stats.ms_phase order: selection, propagation,
          // organization, events
          const int from[4] = {0, 2, 1, 3}, to[4] = {1, 3, 2, 4};
          for (int q = 0; q < 4; ++q) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[from[q]], ev[to[q]]));
            phase_ms[q] += ms;
          }
          timed_rounds++;
          prop_n += fused ? 1 : o.hops;
        }
      }
      {
        const u64 ran = host_ctl.round - rounds_before;
        const u64 n_now = host_ctl.cnt[C_N];
        chunk = o.rounds_per_sync;
        if (ran > 0 && n_prev > n_now) {
          const double rate = (double)(n_prev - n_now) / (double)ran;
          const double left = (double)n_now / rate + 1.0;
          if (left < (double)chunk) chunk = left < 2.0 ? 2 : (int)left;
        }
        n_prev = n_now;
      }
      rounds_before = host_ctl.round;
      if (!strided && fused_blocks == 0)
        pool_blocks = grid_for(std::max<int64_t>(2 * (int64_t)host_ctl.peak, 2 * o.k), 1024);
      if (host_ctl.badidx)
        return set_err(PCH_EDEVICE, "a window or event named a half-edge or vertex outside the mesh");
      if (host_ctl.overflow) {
        overflow = true;
        break;
      }
      if (host_ctl.done) break;
      if ((int64_t)host_ctl.round > kMaxRounds)
        return set_err(PCH_EOVERFLOW, "no termination after the maximum number of rounds");
    }
    if (!overflow) break;
    if (o.pool_limit > 0 && cap >= o.pool_limit)
      return set_err(PCH_EOVERFLOW, "window pool exceeded pool_limit");
    cap *= 2;
    if (o.pool_limit > 0 && cap > o.pool_limit) cap = o.pool_limit;
    restarts++;
  }
  if (host_ctl.nonfinite) return set_err(PCH_ENUMERIC, "non-finite apex crossing in a window");
  // distances out (bit patterns are the doubles)
  HIP_TRY(hipMemcpyAsync(dist, M->g, sizeof(double) * H.nv, hipMemcpyDeviceToDevice, st));
  M->last_rounds = (int64_t)host_ctl.round;
  if (o.collect_stats) {
    const int64_t n = std::min<int64_t>(M->last_rounds, M->w.dlog_cap);
    M->last_log.assign((size_t)n * C_NUM, 0);
    if (n) HIP_TRY(hipMemcpyAsync(M->last_log.data(), M->w.dlog, sizeof(int64_t) * n * C_NUM, hipMemcpyDeviceToHost, st));
  } else {
    M->last_log.clear();
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (stats) {
    const u64* T = host_ctl.tot;
    stats->rounds = (int64_t)host_ctl.round;
    stats->created = (int64_t)(T[C_KIDS] + T[C_FANWIN]);
    stats->processed = (int64_t)T[C_SEL];
    stats->stale = (int64_t)T[C_STALE];
    stats->tiny = (int64_t)T[C_TINY];
    stats->ich_dropped = (int64_t)T[C_ICH];
    stats->dist_events = (int64_t)T[C_DEV];
    stats->angle_events = (int64_t)T[C_AEV];
    stats->fans = (int64_t)T[C_FANS];
    stats->fan_windows = (int64_t)T[C_FANWIN];
    stats->deferred = (int64_t)T[C_DEFER];
    stats->peak_pool = (int64_t)host_ctl.peak;
    stats->restarts = restarts;
    stats->ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    stats->ms_propagate = phase_ms[1];
    for (int q = 0; q < 4; ++q) stats->ms_phase[q] = phase_ms[q];
    stats->timed_rounds = timed_rounds;
    stats->propagate_launches = prop_n;
    stats->hop_launches = (o.fuse_hops != 0 && o.hops <= kFuseHops) ? 1 : o.hops;
    stats->pool_windows = (int64_t)T[C_N];
    stats->selected = (int64_t)host_ctl.xcnt[X_SEL1];
    stats->scan_fused = plan_used == kScanFusedReg ? 2 : (plan_used == kScanFused ? 1 : 0);
    stats->fused_workgroups = fused_wg;
    stats->delta0 = delta0;
  }
  return PCH_OK;
}

pch_status pch_geodesic(pch_mesh M, const int32_t* sources, int32_t m, double* dist, void* hip_stream,
                        const pch_options* opts, pch_stats* stats) {
  return geodesic_core(M, sources, m, dist, hip_stream, opts, stats, nullptr);
}

}  // extern "C"

namespace {

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
pch_status noalloc_scratch(ScratchArena* out) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static void* ptr[kMaxDev] = {};
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDev) return set_err(PCH_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_err(PCH_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    ptr[dev] = p;
  }
  *out = ScratchArena{static_cast<char*>(ptr[dev]), kScratchBytes};
  return PCH_OK;
}

}  // namespace

extern "C" {

pch_status pch_geodesic_noalloc(pch_mesh M, const int32_t* sources, int32_t m, double* dist, void* hip_stream,
                                const pch_options* opts, pch_stats* stats) {
  if (!M || !sources || !dist) return set_err(PCH_EINVAL, "null pointer argument");
  ScratchArena arena;
  const pch_status s = noalloc_scratch(&arena);
  if (s != PCH_OK) return s;
  return geodesic_core(M, sources, m, dist, hip_stream, opts, stats, &arena);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched fields (host)
// ---------------------------------------------------------------------------

struct pch_batch_s {
  std::vector<pch_mesh> meshes;
  std::vector<int32_t> fmesh, fsrc;
  std::vector<int64_t> off;  // n_fields + 1
  std::vector<int32_t> order;
  std::vector<u64> cost;  // expected workgroup time per field: the last run's, else 24 per half-edge
  std::vector<u64> wins;  // expected windows per field: the last run's, else 24 per half-edge
  std::vector<double> delta0;
  pch_batch_options o;
  int device = 0;
  int n_cu = 0;
  int n_teams = 0;
  int64_t max_nv = 0, max_nh = 0;
  BatchDev B{};
  // device tables
  DevMesh* d_meshes = nullptr;
  int64_t *d_nv = nullptr, *d_nh = nullptr, *d_off = nullptr, *d_fstat = nullptr;
  double* d_delta0 = nullptr;
  int32_t *d_fmesh = nullptr, *d_fsrc = nullptr, *d_order = nullptr;
  u64 *d_cost = nullptr, *d_wins = nullptr;
  u64* d_queue = nullptr;
  int64_t* d_fn = nullptr;  // vertices per field (learned cutoff tables)
  u32* d_cdf = nullptr;     // LEARNED: [n_fields][kCdfBins + 1]
  double* d_pbin = nullptr; // LEARNED: [n_fields]
  GangRec* d_gang = nullptr;
  u32* d_board = nullptr;
  bool slots = false;
  hipStream_t stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  double* g_out = nullptr;
  std::vector<int64_t> fstat;
};

namespace {

void free_slots(pch_batch_s* b) {
  if (!b->slots) return;
  BatchDev& B = b->B;
  for (void* p : {(void*)B.pbb, (void*)B.ppp, (void*)B.psk, (void*)B.pes, (void*)B.ev_vq, (void*)B.ev_d, (void*)B.ev_xy, (void*)B.ae_e, (void*)B.ae_D,
                  (void*)B.ae_X, (void*)B.g, (void*)B.fanth, (void*)B.claim, (void*)B.as, (void*)B.gw,
                  (void*)B.asw})
    (void)hipFree(p);
  b->slots = false;
}

void drop_graph(pch_batch_s* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  b->g_out = nullptr;
}

// Longest expected field first (longest processing time first).
void sort_by_cost(pch_batch_s* b) {
  const int nf = (int)b->cost.size();
  b->order.resize(nf);
  for (int f = 0; f < nf; ++f) b->order[f] = f;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return b->cost[x] > b->cost[y]; });
}

// (Re)allocates the per-workgroup buffers for the current options.
pch_status alloc_slots(pch_batch_s* b) {
  free_slots(b);
  drop_graph(b);
  BatchDev& B = b->B;
  const int nf = (int)b->fmesh.size();
  // without helpers a workgroup per field at most; with them every resident
  // slot, since the spare workgroups share the running fields
  const int slots = b->o.teams_per_cu * b->n_cu;
  b->n_teams = std::max(1, b->o.gang > 1 ? slots : std::min(nf, slots));
  int64_t cap = b->o.pool_capacity;
  // a team's pool holds at least three rounds' worth of windows (3 k)
  if (cap <= 0) cap = std::min<int64_t>(std::max<int64_t>({32768, b->max_nh / 12, 3 * b->o.k}), 1 << 21);
  B.cap = cap;
  B.ecap = cap;
  B.acap = std::max<int64_t>(cap / 2, 1024);
  // buffers for the workgroups that may lead a field: one per field at most
  const int64_t T = std::min<int64_t>(b->n_teams, nf);
  B.n_store = (int32_t)T;
  B.hops = b->o.hops;
  B.nslot = B.hops > 1 ? 5 : 3;
  const int64_t np = T * B.nslot * B.cap, ne = T * 3 * B.ecap, na = T * B.acap;
  HIP_TRY(dalloc(&B.pbb, np));
  HIP_TRY(dalloc(&B.ppp, np));
  HIP_TRY(dalloc(&B.psk, np));
  HIP_TRY(dalloc(&B.pes, np));
  HIP_TRY(dalloc(&B.ev_vq, ne));
  HIP_TRY(dalloc(&B.ev_d, ne));
  HIP_TRY(dalloc(&B.ev_xy, ne));
  HIP_TRY(dalloc(&B.ae_e, na));
  HIP_TRY(dalloc(&B.ae_D, na));
  HIP_TRY(dalloc(&B.ae_X, na));
  HIP_TRY(dalloc(&B.g, T * b->max_nv));
  HIP_TRY(dalloc(&B.gw, T * b->max_nv));
  HIP_TRY(dalloc(&B.asw, T * b->max_nh));
  HIP_TRY(dalloc(&B.fanth, T * b->max_nv));
  HIP_TRY(dalloc(&B.claim, T * b->max_nv));
  HIP_TRY(dalloc(&B.as, T * b->max_nh));
  b->slots = true;
  B.gang_max = b->o.gang;
  B.wait = b->o.wait_ticks > 0 ? (u64)b->o.wait_ticks : kGangWait;
  B.max_nv = b->max_nv;
  B.max_nh = b->max_nh;
  B.k = b->o.k;
  B.eps = b->o.eps_tiny;
  B.ch_on = (b->o.filters & 1) != 0;
  B.ich_on = (b->o.filters & 2) != 0;
  B.full_fan = (b->o.filters & 4) != 0;
  B.retest = (b->o.filters & 8) != 0;
  return PCH_OK;
}

void enqueue_batch(pch_batch_s* b, hipStream_t st) {
  const int nr = std::max<int>((int)b->fmesh.size(), kMaxXcc * kBoard);
  k_batch_reset<<<(nr + 255) / 256, 256, 0, st>>>(b->B);
  if (b->o.team_threads == 1024)
    k_batch<1024><<<b->n_teams, 1024, 0, st>>>(b->B);
  else if (b->o.team_threads == 512)
    k_batch<512><<<b->n_teams, 512, 0, st>>>(b->B);
  else
    k_batch<kBlock><<<b->n_teams, kBlock, 0, st>>>(b->B);
}

// One run of the batch into out (graph replay when enabled), then reruns of
// the fields that did not finish in a workgroup.
pch_status batch_run(pch_batch_s* b, double* out, hipStream_t user, pch_batch_stats* stats) {
  auto t_start = std::chrono::steady_clock::now();
  HIP_TRY(hipStreamSynchronize(user));
  b->B.out = out;
  const int nf = (int)b->fmesh.size();
  // the processing order and expected costs of this run (outside the graph)
  HIP_TRY(hipMemcpyAsync(b->d_order, b->order.data(), sizeof(int32_t) * nf, hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_cost, b->cost.data(), sizeof(u64) * nf, hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_wins, b->wins.data(), sizeof(u64) * nf, hipMemcpyHostToDevice, b->stream));
  if (b->o.select_mode == PCH_SELECT_LEARNED) {
    // every field's predicted-distance table, from the predictions as they
    // are now (outside the graph)
    enqueue_pred_cdf(PredFields{b->o.predicted, b->d_off, b->d_fn, 0, nf, b->d_cdf, b->d_pbin}, b->stream);
    std::vector<double> pb(nf);
    HIP_TRY(hipMemcpyAsync(pb.data(), b->d_pbin, sizeof(double) * nf, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (int f = 0; f < nf; ++f)
      if (!(pb[f] > 0.0)) return set_err(PCH_EINVAL, "predicted distances must be positive");
  }
  if (b->o.use_graph) {
    if (!b->gexec || b->g_out != out) {
      drop_graph(b);
      hipGraph_t graph;
      HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      enqueue_batch(b, b->stream);
      HIP_TRY(hipStreamEndCapture(b->stream, &graph));
      hipError_t e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return set_err(PCH_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      b->g_out = out;
    }
    HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
  } else {
    enqueue_batch(b, b->stream);
    HIP_TRY(hipGetLastError());
  }
  b->fstat.assign((size_t)nf * kFieldStat, 0);
  HIP_TRY(hipMemcpyAsync(b->fstat.data(), b->d_fstat, sizeof(int64_t) * nf * kFieldStat, hipMemcpyDeviceToHost,
                         b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  int64_t reruns = 0;
  for (int f = 0; f < nf; ++f) {
    int64_t* fs = &b->fstat[(size_t)f * kFieldStat];
    if (fs[0] == 0) continue;
    pch_options o;
    pch_options_default(&o);
    o.select_mode = b->o.select_mode;
    if (o.select_mode == PCH_SELECT_LEARNED) {
      o.predicted = b->o.predicted + b->off[f];
      o.w0 = b->o.w0;
    }
    o.k = b->o.k;
    o.delta0 = b->delta0[b->fmesh[f]];
    o.filters = b->o.filters;
    o.eps_tiny = b->o.eps_tiny;
    o.hops = b->o.hops;
    pch_stats s1;
    pch_status rc = pch_geodesic(b->meshes[b->fmesh[f]], &b->fsrc[f], 1, out + b->off[f], b->stream, &o, &s1);
    if (rc != PCH_OK) return rc;
    fs[1] = s1.rounds;
    fs[2] = s1.processed;
    fs[3] = s1.created;
    fs[4] = s1.fans;
    fs[5] = s1.peak_pool;
    fs[6] = s1.stale;
    fs[7] = 0;
    fs[8] = 0;
    fs[9] = 0;
    reruns++;
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  // The next run orders and shares the fields by what they took now: the
  // workgroup time of leader and helpers and the windows (a rerun field
  // keeps its time at the batch's time per window).
  {
    double tk = 0.0, wn = 0.0;
    for (int f = 0; f < nf; ++f) {
      const int64_t* fs = &b->fstat[(size_t)f * kFieldStat];
      if (fs[7] > 0) {
        tk += (double)(fs[7] + fs[9]);
        wn += (double)fs[2];
      }
    }
    const double per_win = wn > 0.0 ? tk / wn : 1.0;
    for (int f = 0; f < nf; ++f) {
      const int64_t* fs = &b->fstat[(size_t)f * kFieldStat];
      b->wins[f] = std::max<u64>(1, (u64)fs[2]);
      b->cost[f] = fs[7] > 0 ? (u64)(fs[7] + fs[9]) : std::max<u64>(1, (u64)(per_win * (double)fs[2]));
    }
  }
  sort_by_cost(b);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->fields = nf;
    stats->reruns = reruns;
    stats->teams = b->n_teams;
    stats->k = b->o.k;
    for (int f = 0; f < nf; ++f) {
      const int64_t* fs = &b->fstat[(size_t)f * kFieldStat];
      stats->max_rounds = std::max(stats->max_rounds, fs[1]);
      stats->processed += fs[2];
      stats->created += fs[3];
    }
    stats->ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  }
  return PCH_OK;
}

}  // namespace

extern "C" {

void pch_batch_options_default(pch_batch_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->k = 1024;
  o->teams_per_cu = 2;
  o->filters = 3;
  o->eps_tiny = 0.0;
  o->pool_capacity = 0;
  o->use_graph = 1;
  o->team_threads = 256;
  o->hops = 1;
  o->gang = 1;
  o->select_mode = PCH_SELECT_DELTA;
  o->predicted = nullptr;
  o->w0 = 4.0;
}

void pch_batch_destroy(pch_batch b) {
  if (!b) return;
  drop_graph(b);
  free_slots(b);
  for (void* p : {(void*)b->d_meshes, (void*)b->d_nv, (void*)b->d_nh, (void*)b->d_off, (void*)b->d_fstat,
                  (void*)b->d_delta0, (void*)b->d_fmesh, (void*)b->d_fsrc, (void*)b->d_order, (void*)b->d_queue,
                  (void*)b->d_gang, (void*)b->d_board, (void*)b->d_cost, (void*)b->d_wins, (void*)b->d_fn,
                  (void*)b->d_cdf, (void*)b->d_pbin})
    (void)hipFree(p);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

pch_status pch_batch_create(const pch_mesh* meshes, int32_t n_meshes, const int32_t* field_mesh,
                            const int32_t* field_source, int32_t n_fields, const pch_batch_options* opts,
                            pch_batch* out) {
  if (!meshes || !field_mesh || !field_source || !out) return set_err(PCH_EINVAL, "null pointer argument");
  *out = nullptr;
  if (n_meshes < 1 || n_fields < 1) return set_err(PCH_EINVAL, "need at least one mesh and one field");
  pch_batch_options o;
  pch_batch_options_default(&o);
  if (opts) o = *opts;
  if (o.hops == 0) o.hops = 1;
  if (o.gang == 0) o.gang = 1;
  if (o.wait_ticks < 0) return set_err(PCH_EINVAL, "bad batch option");
  if (o.k < 1 || o.teams_per_cu < 1 || !(o.eps_tiny >= 0.0) || (o.team_threads != 256 && o.team_threads != 512 && o.team_threads != 1024) ||
      o.hops < 1 || o.hops > kMaxHops || o.gang < 1 || o.gang > kMaxGang)
    return set_err(PCH_EINVAL, "bad batch option");
  if (o.select_mode != PCH_SELECT_DELTA && o.select_mode != PCH_SELECT_LEARNED)
    return set_err(PCH_EINVAL, "batched fields take the adaptive step or the learned cutoff");
  if (o.select_mode == PCH_SELECT_LEARNED && !o.predicted)
    return set_err(PCH_EINVAL, "learned selection needs predicted distances");
  if (!(o.w0 >= 0.0)) return set_err(PCH_EINVAL, "bad batch option");
  if (o.w0 == 0.0) o.w0 = 4.0;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  for (int i = 0; i < n_meshes; ++i) {
    if (!meshes[i]) return set_err(PCH_EINVAL, "null mesh in batch");
    if (meshes[i]->device != dev) return set_err(PCH_EINVAL, "mesh was created on another device");
  }
  for (int f = 0; f < n_fields; ++f) {
    if (field_mesh[f] < 0 || field_mesh[f] >= n_meshes) return set_err(PCH_EINVAL, "field mesh index out of range");
    if (field_source[f] < 0 || field_source[f] >= meshes[field_mesh[f]]->host.nv)
      return set_err(PCH_EINVAL, "field source vertex out of range");
  }
  pch_batch_s* b = new (std::nothrow) pch_batch_s();
  if (!b) return set_err(PCH_ENOMEM, "host allocation failed");
  struct Guard {
    pch_batch_s*& b;
    ~Guard() {
      if (b) pch_batch_destroy(b);
    }
  } guard{b};
  b->meshes.assign(meshes, meshes + n_meshes);
  b->fmesh.assign(field_mesh, field_mesh + n_fields);
  b->fsrc.assign(field_source, field_source + n_fields);
  b->o = o;
  b->device = dev;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  b->n_cu = prop.multiProcessorCount;
  HIP_TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  std::vector<DevMesh> dm(n_meshes);
  std::vector<int64_t> nv(n_meshes), nh(n_meshes);
  b->delta0.resize(n_meshes);
  for (int i = 0; i < n_meshes; ++i) {
    pch_mesh_s* M = meshes[i];
    dm[i] = DevMesh{M->hl,    M->phi,    M->alpha, M->twin, M->hv, M->theta, M->flags, M->coff,
                    M->corner, M->crec, (int32_t)M->host.nv, (int32_t)M->host.nh};
    nv[i] = M->host.nv;
    nh[i] = M->host.nh;
    double sum = 0.0;
    for (int64_t j = 0; j < M->host.nh; ++j) sum += M->host.he[j].L;
    b->delta0[i] = 2.0 * (sum / (double)M->host.nh);
    b->max_nv = std::max(b->max_nv, nv[i]);
    b->max_nh = std::max(b->max_nh, nh[i]);
  }
  b->off.resize(n_fields + 1);
  b->off[0] = 0;
  for (int f = 0; f < n_fields; ++f) b->off[f + 1] = b->off[f] + nv[field_mesh[f]];
  b->cost.resize(n_fields);
  b->wins.resize(n_fields);
  for (int f = 0; f < n_fields; ++f) b->cost[f] = b->wins[f] = 24 * (u64)nh[field_mesh[f]];
  sort_by_cost(b);
  HIP_TRY(dalloc(&b->d_meshes, n_meshes));
  HIP_TRY(dalloc(&b->d_nv, n_meshes));
  HIP_TRY(dalloc(&b->d_nh, n_meshes));
  HIP_TRY(dalloc(&b->d_delta0, n_meshes));
  HIP_TRY(dalloc(&b->d_fmesh, n_fields));
  HIP_TRY(dalloc(&b->d_fsrc, n_fields));
  HIP_TRY(dalloc(&b->d_off, n_fields));
  HIP_TRY(dalloc(&b->d_order, n_fields));
  HIP_TRY(dalloc(&b->d_cost, n_fields));
  HIP_TRY(dalloc(&b->d_wins, n_fields));
  HIP_TRY(dalloc(&b->d_fstat, (int64_t)n_fields * kFieldStat));
  HIP_TRY(dalloc(&b->d_queue, 2));
  HIP_TRY(dalloc(&b->d_gang, n_fields));
  HIP_TRY(dalloc(&b->d_board, kMaxXcc * kBoard));
  HIP_TRY(hipMemcpy(b->d_meshes, dm.data(), sizeof(DevMesh) * n_meshes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_nv, nv.data(), sizeof(int64_t) * n_meshes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_nh, nh.data(), sizeof(int64_t) * n_meshes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_delta0, b->delta0.data(), sizeof(double) * n_meshes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_fmesh, field_mesh, sizeof(int32_t) * n_fields, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_fsrc, field_source, sizeof(int32_t) * n_fields, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_off, b->off.data(), sizeof(int64_t) * n_fields, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_order, b->order.data(), sizeof(int32_t) * n_fields, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_cost, b->cost.data(), sizeof(u64) * n_fields, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(b->d_wins, b->wins.data(), sizeof(u64) * n_fields, hipMemcpyHostToDevice));
  BatchDev& B = b->B;
  B.meshes = b->d_meshes;
  B.mesh_nv = b->d_nv;
  B.mesh_nh = b->d_nh;
  B.mesh_delta0 = b->d_delta0;
  B.field_mesh = b->d_fmesh;
  B.field_src = b->d_fsrc;
  B.field_off = b->d_off;
  B.order = b->d_order;
  B.cost = b->d_cost;
  B.wins = b->d_wins;
  B.n_fields = n_fields;
  B.fstat = b->d_fstat;
  B.queue = b->d_queue;
  B.gang = b->d_gang;
  B.board = b->d_board;
  B.max_rounds = kMaxRounds;
  B.mode = o.select_mode;
  B.w0 = o.w0;
  if (o.select_mode == PCH_SELECT_LEARNED) {
    std::vector<int64_t> fn(n_fields);
    for (int f = 0; f < n_fields; ++f) fn[f] = nv[field_mesh[f]];
    HIP_TRY(dalloc(&b->d_fn, n_fields));
    HIP_TRY(dalloc(&b->d_cdf, (int64_t)n_fields * (kCdfBins + 1)));
    HIP_TRY(dalloc(&b->d_pbin, n_fields));
    HIP_TRY(hipMemcpy(b->d_fn, fn.data(), sizeof(int64_t) * n_fields, hipMemcpyHostToDevice));
    B.cdf = b->d_cdf;
    B.pbin = b->d_pbin;
  }
  pch_status s = alloc_slots(b);
  if (s != PCH_OK) return s;
  *out = b;
  b = nullptr;  // owned by the caller now
  return PCH_OK;
}

pch_status pch_batch_offsets(pch_batch b, int64_t* offsets) {
  if (!b || !offsets) return set_err(PCH_EINVAL, "null pointer argument");
  std::memcpy(offsets, b->off.data(), sizeof(int64_t) * b->off.size());
  return PCH_OK;
}

pch_status pch_batch_run(pch_batch b, double* dist, void* hip_stream, pch_batch_stats* stats) {
  if (!b || !dist) return set_err(PCH_EINVAL, "null pointer argument");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != b->device) return set_err(PCH_EINVAL, "batch was created on another device");
  return batch_run(b, dist, (hipStream_t)hip_stream, stats);
}

pch_status pch_batch_field_stats(pch_batch b, int64_t* out) {
  if (!b || !out) return set_err(PCH_EINVAL, "null pointer argument");
  if (b->fstat.empty()) return set_err(PCH_EINVAL, "batch has not run");
  std::memcpy(out, b->fstat.data(), sizeof(int64_t) * b->fstat.size());
  return PCH_OK;
}

}  // extern "C"

namespace {

// Tuner results by batch size bucket: floor(log2) of the largest mesh's
// half-edges, of the half-edges summed over the fields, and of the field
// count, on one GPU architecture. Held for the process; saved to and loaded
// from a text file by pch_tune_cache_save / pch_tune_cache_load.
struct TuneKey {
  std::string arch;
  int max_nh, total_nh, fields;
  bool operator<(const TuneKey& o) const {
    return std::tie(arch, max_nh, total_nh, fields) < std::tie(o.arch, o.max_nh, o.total_nh, o.fields);
  }
};
struct TuneVal {
  int64_t k;
  int32_t team_threads, teams_per_cu, hops, gang;
  double ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

int ilog2(int64_t x) {
  int b = 0;
  while (x > 1) {
    x >>= 1;
    ++b;
  }
  return b;
}

pch_status tune_key(pch_batch_s* b, TuneKey* key) {
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, b->device));
  int64_t total = 0;
  for (int32_t mi : b->fmesh) total += b->meshes[mi]->host.nh;
  *key = TuneKey{std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':')),
                 ilog2(b->max_nh), ilog2(total), ilog2((int64_t)b->fmesh.size())};
  return PCH_OK;
}

}  // namespace

extern "C" {

pch_status pch_batch_tune(pch_batch b, double* dist, void* hip_stream, pch_batch_options* chosen) {
  if (!b || !dist) return set_err(PCH_EINVAL, "null pointer argument");
  const int64_t ks[] = {8192, 16384, 32768, 65536};
  const int shapes[][2] = {{256, 1}, {512, 1}, {1024, 1}};  // team threads, teams per CU
  const int hop_set[] = {1, 4};
  const int gangs[] = {1, 2, 4, 16};
  pch_batch_options best = b->o;
  double best_ms = INFINITY;
  auto trial = [&]() -> pch_status {
    pch_status s = alloc_slots(b);
    if (s != PCH_OK) return s;
    pch_batch_stats st;
    s = batch_run(b, dist, (hipStream_t)hip_stream, &st);
    if (s != PCH_OK) return s;
    if (st.ms_total < best_ms) {
      best_ms = st.ms_total;
      best = b->o;
    }
    return PCH_OK;
  };
  // k, workgroup shape and hops with up to 8 workgroups per field, then the
  // gang size at the best of those
  for (const auto& sh : shapes) {
    for (int64_t k : ks) {
      for (int hops : hop_set) {
        b->o.k = k;
        b->o.team_threads = sh[0];
        b->o.teams_per_cu = sh[1];
        b->o.hops = hops;
        b->o.gang = 8;
        pch_status s = trial();
        if (s != PCH_OK) return s;
      }
    }
  }
  for (int gang : gangs) {
    b->o = best;
    b->o.gang = gang;
    pch_status s = trial();
    if (s != PCH_OK) return s;
  }
  b->o = best;
  pch_status s = alloc_slots(b);
  if (s != PCH_OK) return s;
  if (chosen) *chosen = best;
  TuneKey key;
  s = tune_key(b, &key);
  if (s != PCH_OK) return s;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[key] = TuneVal{best.k, best.team_threads, best.teams_per_cu, best.hops, best.gang, best_ms};
  return PCH_OK;
}

pch_status pch_batch_tune_cached(pch_batch b, double* dist, void* hip_stream, pch_batch_options* chosen,
                                 int32_t* hit) {
  if (!b || !dist) return set_err(PCH_EINVAL, "null pointer argument");
  TuneKey key;
  pch_status s = tune_key(b, &key);
  if (s != PCH_OK) return s;
  bool found = false;
  TuneVal v{};
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      found = true;
      v = it->second;
    }
  }
  if (hit) *hit = found ? 1 : 0;
  if (!found) return pch_batch_tune(b, dist, hip_stream, chosen);
  b->o.k = v.k;
  b->o.team_threads = v.team_threads;
  b->o.teams_per_cu = v.teams_per_cu;
  b->o.hops = v.hops;
  b->o.gang = v.gang;
  s = alloc_slots(b);
  if (s != PCH_OK) return s;
  if (chosen) *chosen = b->o;
  return PCH_OK;
}

pch_status pch_tune_cache_save(const char* path) {
  if (!path) return set_err(PCH_EINVAL, "null pointer argument");
  FILE* f = std::fopen(path, "w");
  if (!f) return set_err(PCH_EINVAL, std::string("cannot write ") + path);
  std::fprintf(f, "# arch max_nh_log2 total_nh_log2 fields_log2 k team_threads teams_per_cu hops gang ms\n");
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const auto& kv : g_tune)
      std::fprintf(f, "%s %d %d %d %lld %d %d %d %d %.3f\n", kv.first.arch.c_str(), kv.first.max_nh,
                   kv.first.total_nh, kv.first.fields, (long long)kv.second.k, kv.second.team_threads,
                   kv.second.teams_per_cu, kv.second.hops, kv.second.gang, kv.second.ms);
  }
  const bool ok = std::fclose(f) == 0;
  return ok ? PCH_OK : set_err(PCH_EINVAL, std::string("cannot write ") + path);
}

pch_status pch_tune_cache_load(const char* path) {
  if (!path) return set_err(PCH_EINVAL, "null pointer argument");
  FILE* f = std::fopen(path, "r");
  if (!f) return set_err(PCH_EINVAL, std::string("cannot read ") + path);
  char line[512];
  int n = 0;
  pch_status rc = PCH_OK;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    char arch[64];
    TuneKey key;
    TuneVal v;
    long long k = 0;
    if (std::sscanf(line, "%63s %d %d %d %lld %d %d %d %d %lf", arch, &key.max_nh, &key.total_nh, &key.fields, &k,
                    &v.team_threads, &v.teams_per_cu, &v.hops, &v.gang, &v.ms) != 10 ||
        k < 1 || (v.team_threads != 256 && v.team_threads != 512 && v.team_threads != 1024) ||
        v.teams_per_cu < 1 || v.hops < 1 || v.hops > kMaxHops || v.gang < 1 || v.gang > kMaxGang) {
      rc = set_err(PCH_EINVAL, std::string("bad line in ") + path);
      break;
    }
    key.arch = arch;
    v.k = k;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = v;
    ++n;
  }
  std::fclose(f);
  return rc;
}

pch_status pch_voronoi(pch_mesh mesh, const int32_t* sources, int32_t m, double* dist, int32_t* label,
                       void* hip_stream, const pch_batch_options* opts) {
  if (!mesh || !sources || !dist || !label) return set_err(PCH_EINVAL, "null pointer argument");
  if (m < 1) return set_err(PCH_EINVAL, "need at least one source");
  const int64_t nv = mesh->host.nv;
  std::vector<int32_t> fmesh(m, 0);
  pch_batch b = nullptr;
  pch_status s = pch_batch_create(&mesh, 1, fmesh.data(), sources, m, opts, &b);
  if (s != PCH_OK) return s;
  double* fields = nullptr;
  hipError_t e = hipMalloc(&fields, sizeof(double) * (size_t)m * (size_t)nv);
  if (e != hipSuccess) {
    pch_batch_destroy(b);
    return set_err(PCH_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  s = pch_batch_run(b, fields, hip_stream, nullptr);
  if (s == PCH_OK) {
    hipStream_t st = (hipStream_t)hip_stream;
    k_voronoi<<<grid_for(nv, 1024), kBlock, 0, st>>>(fields, m, nv, dist, label);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = set_err(PCH_EDEVICE, std::string("voronoi: ") + hipGetErrorString(e));
  }
  (void)hipFree(fields);
  pch_batch_destroy(b);
  return s;
}

}  // extern "C"
