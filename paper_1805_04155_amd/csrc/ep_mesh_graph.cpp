// Host construction of the mesh graph (see ep_mesh_graph.h): the integer
// structures behind the assembly of Section 6 (the pattern MATLAB's sparse
// builds implicitly) and the colour rounds of the deterministic scatter.
#include "ep_mesh_graph.h"

#include <algorithm>
#include <numeric>
#include <thread>

namespace ep {
namespace {

template <class F>
void parallel_for(int64_t n, F f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096) nt = 1;
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=] { f(a, b); });
  }
  for (auto &x : th) x.join();
}

}  // namespace

std::string build_mesh_graph(int64_t n_n, int64_t n_e, int n_p, int dim, const int32_t *E,
                             bool sorted_columns, int64_t chunk, int max_colours, MeshGraph &g) {
  for (int64_t i = 0; i < n_e * n_p; ++i)
    if (E[i] < 0 || E[i] >= n_n) return "node id out of range in elem";
  // the nodes of an element are distinct (the assembly ranks them)
  for (int64_t e = 0; e < n_e; ++e) {
    const int32_t *en = E + e * n_p;
    for (int i = 0; i < n_p; ++i)
      for (int j = i + 1; j < n_p; ++j)
        if (en[i] == en[j]) return "repeated node in an element";
  }
  // node -> (element, local node), ascending element
  g.n2e_ptr.assign(n_n + 1, 0);
  g.n2e.assign(n_e * n_p, 0);
  g.fslot.assign(n_e * n_p, 0);
  g.slot_elem.assign(n_e * n_p, 0);
  for (int64_t i = 0; i < n_e * n_p; ++i) g.n2e_ptr[E[i] + 1]++;
  for (int64_t m = 0; m < n_n; ++m) g.n2e_ptr[m + 1] += g.n2e_ptr[m];
  {
    std::vector<int32_t> fill(g.n2e_ptr.begin(), g.n2e_ptr.end() - 1);
    for (int64_t e = 0; e < n_e; ++e)
      for (int p = 0; p < n_p; ++p) {
        const int32_t k = fill[E[e * n_p + p]]++;
        g.n2e[k] = (int32_t)(e * n_p + p);
        g.fslot[e * n_p + p] = k;  // element force vectors are stored node by node
        g.slot_elem[k] = (int32_t)e;
      }
  }
  // node adjacency -> node-block CSR
  const std::vector<int32_t> &n2e_ptr = g.n2e_ptr, &n2e = g.n2e;
  std::vector<int32_t> deg(n_n, 0);
  auto neighbours = [&](int64_t m, std::vector<int32_t> &mark, std::vector<int32_t> &lst) {
    lst.clear();
    for (int k = n2e_ptr[m]; k < n2e_ptr[m + 1]; ++k) {
      const int64_t e = n2e[k] / n_p;
      for (int p = 0; p < n_p; ++p) {
        const int32_t v = E[e * n_p + p];
        if (mark[v] != (int32_t)m) {
          mark[v] = (int32_t)m;
          lst.push_back(v);
        }
      }
    }
    std::sort(lst.begin(), lst.end());
  };
  parallel_for(n_n, [&](int64_t a, int64_t b) {
    std::vector<int32_t> mark(n_n, -1), lst;
    for (int64_t m = a; m < b; ++m) {
      neighbours(m, mark, lst);
      deg[m] = (int32_t)lst.size();
    }
  });
  int64_t nnzb = 0;
  for (int64_t m = 0; m < n_n; ++m) nnzb += deg[m];
  if (nnzb * dim * dim >= (int64_t)1 << 31) return "matrix too large for 32-bit indices";
  g.nnzb = nnzb;
  g.bptr.assign(n_n + 1, 0);
  for (int64_t m = 0; m < n_n; ++m) g.bptr[m + 1] = g.bptr[m] + deg[m];
  g.bcol.assign(nnzb, 0);
  g.bdiag.assign(n_n, 0);
  parallel_for(n_n, [&](int64_t a, int64_t b) {
    std::vector<int32_t> mark(n_n, -1), lst;
    for (int64_t m = a; m < b; ++m) {
      neighbours(m, mark, lst);
      std::copy(lst.begin(), lst.end(), g.bcol.begin() + g.bptr[m]);
      g.bdiag[m] = (int32_t)(g.bptr[m] + (std::lower_bound(lst.begin(), lst.end(), (int32_t)m) -
                                          lst.begin()));
    }
  });
  // element position map of node pairs
  g.bpos.assign((size_t)n_e * n_p * n_p, 0);
  parallel_for(n_e, [&](int64_t a, int64_t b) {
    for (int64_t e = a; e < b; ++e)
      for (int p = 0; p < n_p; ++p) {
        const int32_t m = E[e * n_p + p];
        const int32_t *lo = g.bcol.data() + g.bptr[m], *hi = g.bcol.data() + g.bptr[m + 1];
        for (int pp = 0; pp < n_p; ++pp) {
          const int32_t *it = std::lower_bound(lo, hi, E[e * n_p + pp]);
          g.bpos[(e * n_p + p) * n_p + pp] = (int32_t)(it - g.bcol.data());
        }
      }
  });
  // position map with each row's columns in ascending global node order
  g.bposs.clear();
  if (sorted_columns) {
    g.bposs.resize((size_t)n_e * n_p * n_p);
    parallel_for(n_e, [&](int64_t a, int64_t b) {
      std::vector<int> ord(n_p);
      for (int64_t e = a; e < b; ++e) {
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(),
                  [&](int x, int y) { return E[e * n_p + x] < E[e * n_p + y]; });
        for (int p = 0; p < n_p; ++p)
          for (int r = 0; r < n_p; ++r)
            g.bposs[(e * n_p + p) * n_p + r] = g.bpos[(e * n_p + p) * n_p + ord[r]];
      }
    });
  }
  // greedy colouring: elements of one colour share no node
  g.colour.assign(n_e, -1);
  int n_col = 0;
  {
    std::vector<uint64_t> used((max_colours + 63) / 64);
    for (int64_t e = 0; e < n_e; ++e) {
      std::fill(used.begin(), used.end(), 0);
      for (int p = 0; p < n_p; ++p) {
        const int32_t m = E[e * n_p + p];
        for (int k = n2e_ptr[m]; k < n2e_ptr[m + 1]; ++k) {
          const int64_t e2 = n2e[k] / n_p;
          if (e2 < e) {
            const int cc = g.colour[e2];
            used[cc >> 6] |= 1ull << (cc & 63);
          }
        }
      }
      int cc = 0;
      while (cc < max_colours && ((used[cc >> 6] >> (cc & 63)) & 1ull)) ++cc;
      if (cc >= max_colours)
        return "colouring needs more than " + std::to_string(max_colours) + " colours";
      g.colour[e] = cc;
      n_col = std::max(n_col, cc + 1);
    }
  }
  g.n_col = n_col;
  g.colour_size.assign(n_col, 0);
  for (int64_t e = 0; e < n_e; ++e) g.colour_size[g.colour[e]]++;
  g.colour_first_chunk.assign(n_col + 1, 0);
  for (int col = 0; col < n_col; ++col)
    g.colour_first_chunk[col + 1] =
        g.colour_first_chunk[col] + (int32_t)((g.colour_size[col] + chunk - 1) / chunk);
  const int64_t n_perm = (int64_t)g.colour_first_chunk[n_col] * chunk;
  g.perm.assign(std::max<int64_t>(n_perm, 1), -1);
  {
    std::vector<int64_t> fill(n_col);
    for (int col = 0; col < n_col; ++col) fill[col] = (int64_t)g.colour_first_chunk[col] * chunk;
    for (int64_t e = 0; e < n_e; ++e) g.perm[fill[g.colour[e]]++] = (int32_t)e;
  }
  return "";
}

}  // namespace ep
