// Test infrastructure only (see pch_oracle.cpp's header): the mesh tables both
// CPU references build from the input, per Section 4.1 (half-edge j of face
// j / 3 runs from F[j] to F[next(j)], next(j) = 3 (j / 3) + (j + 1) % 3) and
// the vertex classes of Section 3 (saddle, boundary). Nothing here computes
// windows: ich.cpp and pch_oracle.cpp each do that with their own code.
#ifndef ORACLE_MESH_H
#define ORACLE_MESH_H

#include <cstdint>
#include <string>
#include <vector>

namespace orc {

enum { OK = 0, EINVAL_ = -1, EMESH = -2 };

// Interior vertices with total angle above 2 pi + kSaddle are saddles.
constexpr double kSaddle = 1e-10;

inline int32_t nxt(int32_t j) { return 3 * (j / 3) + (j + 1) % 3; }
inline int32_t prv(int32_t j) { return 3 * (j / 3) + (j + 2) % 3; }

struct OMesh {
  int64_t nv = 0, nf = 0;
  std::vector<int32_t> F;      // start vertex of half-edge j
  std::vector<double> L;       // length of half-edge j
  std::vector<int32_t> twin;   // opposite half-edge or -1
  std::vector<double> ax, ay;  // opposite vertex in j's frame (start at 0, end at (L,0))
  std::vector<double> alpha;   // corner angle at the start of j inside face(j)
  std::vector<double> phi;     // angular position of j around its start vertex
  std::vector<double> theta;   // total angle per vertex
  std::vector<uint8_t> bnd, pseudo;
  std::vector<int32_t> coff, corner;  // CCW list of outgoing half-edges per vertex
};

// Records msg as the calling thread's error text and returns code.
int fail(int code, const std::string& msg);
const char* last_error();

int build_mesh(const int32_t* faces, int64_t nf, int64_t nv, const double* len, OMesh& M);

// Sources sorted and without duplicates; EINVAL_ when empty or out of range.
int sorted_sources(const int32_t* src, int32_t m, int64_t nv, std::vector<int32_t>& out);

}  // namespace orc

#endif
