// Internal declarations shared by the host mesh builder and the device driver
// of the PCH library. Not part of the public C ABI (include/pch.h).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pch {

// Per-half-edge record used by the propagation kernel: everything a window on
// half-edge e needs to unfold across face(e), packed in one 64-byte line.
// Frame of e: start vertex at (0, 0), end vertex at (L, 0), opposite vertex
// at (x2, y2) with y2 > 0 (Section 3, Figure 2).
struct alignas(64) HalfEdge {
  double L;    // |v0 v1|
  double x2;   // opposite vertex v2 in e's frame
  double y2;
  double l02;  // |v0 v2| = length of prev(e)
  double l12;  // |v1 v2| = length of next(e)
  int32_t v0, v1, v2;
  int32_t tl;  // twin(prev(e)): half-edge v0 -> v2 in the face across
  int32_t tr;  // twin(next(e)): half-edge v2 -> v1 in the face across
  int32_t pflags;  // bits 0, 1, 2: v0, v1, v2 is a pseudo-source vertex
};
static_assert(sizeof(HalfEdge) == 64, "half-edge record must be 64 bytes");

// Per-half-edge constants of the propagation beyond the frame itself.
// th0, th1, th2: the angular positions a window on half-edge e needs for the
// incoming angle of its distance events (only read when the vertex is a
// pseudo-source): around v0 the position of e, around v1 the position of
// v1 -> v0 (that of next(e) plus its corner angle), around v2 the position of
// prev(e). (ulx, uly) = (x2, y2) / l02 and (urx, ury) = (L - x2, -y2) / l12:
// the unit vectors along the two edges a window's children live on.
struct alignas(64) HalfEdgeAng {
  double th0, th1, th2;
  double ulx, uly, urx, ury;
  double pad;
};
static_assert(sizeof(HalfEdgeAng) == 64, "half-edge constant record must be 64 bytes");

// Everything a fan needs about one corner of a vertex v (outgoing half-edge
// j = v -> a, face (v, a, b)), stored in CCW order per vertex so that a fan
// reads one record per corner.
struct alignas(32) Corner {
  double alpha;   // corner angle at v
  double phi;     // angular position of j around v
  double l_va;    // |v a| = length of j
  double l_vb;    // |v b| = length of prev(j)
  double L;       // |a b| = length of next(j), the edge opposite v
  double x2, y2;  // v in the frame of next(j) (a at 0, b at (L, 0))
  double th_a;    // angular position at a of the direction a -> v
  double th_b;    // angular position at b of the direction b -> v
  int32_t a, b;
  int32_t tw;     // twin(next(j)): the half-edge a fan window lives on, or -1
  int32_t last;   // 1 when v -> b is a boundary edge (j is v's last corner)
};
static_assert(sizeof(Corner) == 96, "corner record must be 96 bytes");

enum : uint8_t { VF_BOUNDARY = 1, VF_PSEUDO = 2 };

struct HostMesh {
  int64_t nv = 0, nf = 0, nh = 0;
  std::vector<HalfEdge> he;      // [nh]
  std::vector<double> phi;       // [nh] angular position of j around its start vertex
  std::vector<double> alpha;     // [nh] corner angle at the start of j
  std::vector<int32_t> twin;     // [nh]
  std::vector<int32_t> hv;       // [nh] start vertex of j
  std::vector<double> theta;     // [nv] total angle
  std::vector<uint8_t> flags;    // [nv] VF_*
  std::vector<int32_t> coff;     // [nv + 1] CSR offsets of the CCW corner lists
  std::vector<int32_t> corner;   // [nh] outgoing half-edges in CCW order
  std::vector<Corner> crec;      // [nh] corner records in the same order
  std::vector<HalfEdgeAng> hang; // [nh]
  int64_t n_boundary_he = 0, n_pseudo = 0;
};

// Builds the mesh tables from faces and half-edge lengths. Returns 0 or a
// negative pch_status; msg receives the reason.
int build_host_mesh(const int32_t* faces, int64_t nf, int64_t nv, const double* he_len, HostMesh& out,
                    std::string& msg);

// Records the thread's last error text (read by pch_last_error) and returns s.
int set_error(int s, const std::string& msg);

// Half-edge lengths from coordinates.
int lengths_from_xyz(const double* xyz, int64_t nv, const int32_t* faces, int64_t nf, std::vector<double>& len,
                     std::string& msg);

}  // namespace pch
