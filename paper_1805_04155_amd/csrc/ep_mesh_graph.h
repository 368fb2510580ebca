// Mesh graph of the hot path, built on the host at setup: the node-to-element
// map, the node-block CSR pattern of K with its diagonal, the element
// position map of node pairs (also in ascending-node column order), a greedy
// element colouring and the colour-major element order.  Plain C++ (no HIP),
// so that it can be built and checked on its own (e.g. under a sanitizer).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace ep {

struct MeshGraph {
  // node m -> slots n2e_ptr[m] .. n2e_ptr[m+1]-1, each holding e * n_p + p
  // (ascending element); fslot[e * n_p + p] is the slot of (e, p) and
  // slot_elem[k] the element of slot k
  std::vector<int32_t> n2e_ptr, n2e, fslot, slot_elem;
  // node-block CSR: row m holds the nodes sharing an element with m,
  // ascending; bdiag[m] is the index of block (m, m)
  std::vector<int32_t> bptr, bcol, bdiag;
  // bpos[e][p][p'] = block index of (node p, node p') of element e; bposs the
  // same with the columns p' taken in ascending global node order
  std::vector<int32_t> bpos, bposs;
  // colour[e]: elements of one colour share no node; colours listed in
  // chunks of `chunk` elements (perm: colour-major, each colour padded to a
  // whole number of chunks with -1), colour_first_chunk[c] its first chunk
  std::vector<int32_t> colour, colour_size, colour_first_chunk, perm;
  int n_col = 0;
  int64_t nnzb = 0;
};

// Builds g for n_e elements of n_p nodes (elem[n_e][n_p], node ids in
// [0, n_n)); dim sizes the 32-bit index check of the scalar non-zeros.
// Returns "" on success, otherwise the reason (invalid connectivity, more
// than max_colours colours, a matrix beyond 32-bit indices).
std::string build_mesh_graph(int64_t n_n, int64_t n_e, int n_p, int dim, const int32_t *elem,
                             bool sorted_columns, int64_t chunk, int max_colours, MeshGraph &g);

}  // namespace ep
