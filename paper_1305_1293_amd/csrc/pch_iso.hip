// Iso-contours of a geodesic distance field, an application on top of the
// exact per-vertex distances (the paper's future work names geodesic Voronoi
// diagrams and other applications that need many exact distances; the
// analytic iso-contours it cites are out of reach once the windows are gone).
// The contour of level c is taken on the piecewise-linear interpolant of the
// vertex distances over each triangle (marching triangles): a face whose
// vertex values are not all on the same side of c (side: d >= c) holds one
// segment, whose endpoints are the points of its two crossing edges where the
// linear interpolant equals c.
//
// Mapping: one thread per (face, level) pair, adjacent threads on the levels
// of the same face; segments are appended with one reservation per wavefront.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "pch.h"
#include "pch_internal.h"

namespace {

using u64 = unsigned long long;
constexpr int kIsoBlock = 256;

struct IsoLevels {
  double v[PCH_ISO_MAX_LEVELS];
};

pch_status iso_err(pch_status s, const std::string& m) { return (pch_status)pch::set_error(s, m); }
#define ISO_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return iso_err(e_ == hipErrorOutOfMemory ? PCH_ENOMEM : PCH_EDEVICE,                  \
                     std::string(#expr) + ": " + hipGetErrorString(e_));                    \
  } while (0)

// Crossing of the level c on the edge from value da to value db (their sides
// differ, so db != da): the fraction of the way from a to b.
__device__ __forceinline__ double crossing(double c, double da, double db) { return (c - da) / (db - da); }

// ctr[0]: segments found (also those beyond cap); ctr[1]: faces with a vertex
// index outside [0, nv).
__global__ void __launch_bounds__(kIsoBlock) k_isolines(const int32_t* __restrict__ faces, int64_t nf, int64_t nv,
                                                        const double* __restrict__ dist, IsoLevels lv, int32_t nl,
                                                        int32_t* __restrict__ seg_he, double* __restrict__ seg_t,
                                                        int32_t* __restrict__ seg_level, int64_t cap, u64* ctr) {
  const int64_t n = nf * nl;
  const int lane = __lane_id();
  for (int64_t i = blockIdx.x * (int64_t)kIsoBlock + threadIdx.x; i - lane < n;
       i += (int64_t)gridDim.x * kIsoBlock) {
    bool has = false;
    int32_t ja = 0, jb = 0, l = 0;
    double ta = 0.0, tb = 0.0;
    if (i < n) {
      const int64_t f = i / nl;
      l = (int32_t)(i - f * nl);
      const int32_t v0 = faces[3 * f], v1 = faces[3 * f + 1], v2 = faces[3 * f + 2];
      const bool ok = v0 >= 0 && v0 < nv && v1 >= 0 && v1 < nv && v2 >= 0 && v2 < nv;
      if (!ok) {
        if (l == 0) atomicAdd(&ctr[1], 1ull);
      } else {
        const double d0 = dist[v0], d1 = dist[v1], d2 = dist[v2];
        // a face with an unreachable vertex has no interpolant
        if (isfinite(d0) && isfinite(d1) && isfinite(d2)) {
          const double c = lv.v[l];
          const bool s0 = d0 >= c, s1 = d1 >= c, s2 = d2 >= c;
          if (!(s0 == s1 && s1 == s2)) {
            // exactly two of the edges 0 (v0 -> v1), 1 (v1 -> v2), 2 (v2 -> v0)
            // cross; the endpoints go in that edge order
            has = true;
            const int32_t j0 = (int32_t)(3 * f);
            if (s0 != s1) {
              ja = j0;
              ta = crossing(c, d0, d1);
              if (s1 != s2) {
                jb = j0 + 1;
                tb = crossing(c, d1, d2);
              } else {
                jb = j0 + 2;
                tb = crossing(c, d2, d0);
              }
            } else {
              ja = j0 + 1;
              ta = crossing(c, d1, d2);
              jb = j0 + 2;
              tb = crossing(c, d2, d0);
            }
          }
        }
      }
    }
    // one reservation per wavefront (every lane of the wavefront is here)
    const u64 mask = __ballot(has);
    if (mask) {
      const int leader = __ffsll((unsigned long long)mask) - 1;
      u64 base = 0;
      if (lane == leader) base = atomicAdd(&ctr[0], (u64)__popcll(mask));
      const unsigned lo = __shfl((unsigned)(base & 0xffffffffull), leader);
      const unsigned hi = __shfl((unsigned)(base >> 32), leader);
      base = ((u64)hi << 32) | lo;
      if (has) {
        const u64 k = base + (u64)__popcll(mask & ((1ull << lane) - 1ull));
        if (k < (u64)cap) {
          seg_he[2 * k] = ja;
          seg_he[2 * k + 1] = jb;
          seg_t[2 * k] = ta;
          seg_t[2 * k + 1] = tb;
          seg_level[k] = l;
        }
      }
    }
  }
}

}  // namespace

extern "C" {

pch_status pch_isolines(const int32_t* faces, int64_t nf, int64_t nv, const double* dist, const double* levels,
                        int32_t n_levels, int32_t* seg_he, double* seg_t, int32_t* seg_level, int64_t cap,
                        int64_t* n_segments, void* hip_stream) {
  if (!n_segments) return iso_err(PCH_EINVAL, "n_segments is NULL");
  *n_segments = 0;
  // half-edge indices 3 f + k are int32
  if (nf < 0 || nv < 1 || nf > (((int64_t)1 << 31) - 1) / 3)
    return iso_err(PCH_EINVAL, "nf must be in [0, (2^31 - 1) / 3], nv >= 1");
  if (n_levels < 1 || n_levels > PCH_ISO_MAX_LEVELS)
    return iso_err(PCH_EINVAL, "n_levels must be in [1, " + std::to_string(PCH_ISO_MAX_LEVELS) + "]");
  if (!levels || (nf > 0 && (!faces || !dist))) return iso_err(PCH_EINVAL, "NULL input");
  if (cap < 0 || (cap > 0 && (!seg_he || !seg_t || !seg_level))) return iso_err(PCH_EINVAL, "bad output buffers");
  IsoLevels lv{};
  for (int i = 0; i < n_levels; ++i) {
    if (!std::isfinite(levels[i])) return iso_err(PCH_EINVAL, "levels must be finite");
    lv.v[i] = levels[i];
  }
  if (nf == 0) return PCH_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  u64* ctr = nullptr;
  ISO_TRY(hipMalloc(&ctr, 2 * sizeof(u64)));
  u64 h[2] = {0, 0};
  hipError_t e = hipMemsetAsync(ctr, 0, 2 * sizeof(u64), st);
  if (e == hipSuccess) {
    const int64_t n = nf * n_levels;
    int64_t blocks = (n + kIsoBlock - 1) / kIsoBlock;
    if (blocks > 4096) blocks = 4096;
    k_isolines<<<(unsigned)blocks, kIsoBlock, 0, st>>>(faces, nf, nv, dist, lv, n_levels, seg_he, seg_t, seg_level,
                                                       cap, ctr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(ctr);
  if (e != hipSuccess)
    return iso_err(e == hipErrorOutOfMemory ? PCH_ENOMEM : PCH_EDEVICE, std::string("pch_isolines: ") +
                                                                            hipGetErrorString(e));
  if (h[1] != 0) return iso_err(PCH_EINVAL, std::to_string(h[1]) + " faces with a vertex index outside [0, nv)");
  *n_segments = (int64_t)h[0];
  if ((int64_t)h[0] > cap)
    return iso_err(PCH_EOVERFLOW, std::to_string(h[0]) + " segments do not fit in " + std::to_string(cap));
  return PCH_OK;
}

}  // extern "C"
