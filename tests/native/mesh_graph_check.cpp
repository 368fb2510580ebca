// Builds the library's host mesh graph (csrc/ep_mesh_graph.cpp) for the
// connectivity of one binary file and writes its arrays to another, so that
// a build with AddressSanitizer / UndefinedBehaviorSanitizer can be driven
// from a test and checked against the oracle's pattern and position map.
//   usage: mesh_graph_check IN OUT
// IN:  int64 n_n, n_e; int32 n_p, dim, sorted; int32 elem[n_e][n_p]
// OUT: int32 status (0 ok, 1 refused: the reason on stderr); then int64
//      nnzb, n_col and the arrays bptr, bcol, bdiag, bpos, bposs (if
//      sorted), colour, n2e_ptr, fslot, slot_elem, perm (int64 length
//      first).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ep_mesh_graph.h"

static void put(FILE *f, const std::vector<int32_t> &v) {
  const int64_t n = (int64_t)v.size();
  fwrite(&n, 8, 1, f);
  if (n) fwrite(v.data(), 4, v.size(), f);
}

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *in = std::fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t sz[2];
  int32_t hdr[3];
  if (std::fread(sz, 8, 2, in) != 2 || std::fread(hdr, 4, 3, in) != 3) return 3;
  std::vector<int32_t> elem((size_t)(sz[1] * hdr[0]));
  if (!elem.empty() && std::fread(elem.data(), 4, elem.size(), in) != elem.size()) return 3;
  std::fclose(in);
  ep::MeshGraph g;
  const std::string why =
      ep::build_mesh_graph(sz[0], sz[1], hdr[0], hdr[1], elem.data(), hdr[2] != 0, 2048, 512, g);
  FILE *out = std::fopen(argv[2], "wb");
  if (!out) return 2;
  const int32_t status = why.empty() ? 0 : 1;
  std::fwrite(&status, 4, 1, out);
  if (!why.empty()) {
    std::fprintf(stderr, "refused: %s\n", why.c_str());
  } else {
    const int64_t nn[2] = {g.nnzb, (int64_t)g.n_col};
    std::fwrite(nn, 8, 2, out);
    for (const auto *v : {&g.bptr, &g.bcol, &g.bdiag, &g.bpos, &g.bposs, &g.colour, &g.n2e_ptr,
                          &g.fslot, &g.slot_elem, &g.perm})
      put(out, *v);
  }
  std::fclose(out);
  return 0;
}
