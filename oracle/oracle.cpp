// oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded CPU implementation of the exact maximum-clique
// method of Rossi, Gleich, Gebremedhin and Patwary (arXiv 1302.6256), written
// from the paper to check the GPU path.  It shares no code, header, table or
// helper with the GPU library.  Only tests, the smoke check and the CPU
// baseline leg of the benchmark may load it; the product never does.
//
// Sections of the paper followed here:
//   Sec. 3 (bounds): core numbers K(v), the degeneracy order, greedy colouring;
//     Fact 1 (omega <= L <= K+1 <= Delta+1), Fact 2 (reduced neighbourhoods).
//   Alg. 1 (HeuristicClique) and Sec. 4.1.
//   Alg. 2 (MaxClique / InitialBranch / Branch) and Secs. 4.2-4.3.
// Readings of places where the paper is silent or ambiguous:
//   R1  Alg. 1 starts the greedy clique of seed v as C = {v}.
//   R2  "decreasing core number order" is decreasing degeneracy rank.
//   R3  the main loop's "smallest reduced degree" order is the static
//       degeneracy rank; a searched vertex is excluded from later
//       neighbourhoods by visiting only higher-ranked neighbours.
//   R4  the neighbourhood-core test of InitialBranch is K(P) < |H|.
//   R6  "Color(P, K_N) in degen. order" colours in reverse local peel order.
//   R7  "natural (any) order" in Branch is increasing rank.
//   R8  Branch picks the largest colour, ties to the latest in colouring order.
//   R10 no periodic rebuild (it cannot change the result).
//   R11 colours are 1..L with no gaps (greedy colouring never skips one).
// The degeneracy rank is the position in (peel round, vertex id) order, where
// peel rounds are the level-synchronous sub-rounds defined in or_peel below.
//
// Parity pins: every exported function is checked in tests/ against closed
// forms, brute force, textbook Bron-Kerbosch, networkx, or invariants of the
// paper's Facts; see the test files named after each function.

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

extern "C" {
int32_t or_peel(int64_t n, const int64_t *off, const int32_t *idx, int32_t *core, int32_t *round,
                int32_t *kmax);
void or_rank(int64_t n, const int32_t *round, int32_t *rank, int32_t *order);
}

namespace {

struct Csr {
  int64_t n;
  const int64_t *off;
  const int32_t *idx;
  int64_t deg(int64_t v) const { return off[v + 1] - off[v]; }
};

// Edge test by binary search in a sorted row.
bool adjacent(const Csr &g, int32_t a, int32_t b) {
  const int32_t *lo = g.idx + g.off[a], *hi = g.idx + g.off[a + 1];
  return std::binary_search(lo, hi, b);
}

// A small graph with an explicit adjacency matrix ("adjacency matrix for
// small graphs", Sec. 4.4), used for neighbourhood subproblems.
struct Local {
  int s = 0;
  std::vector<uint8_t> a;
  bool adj(int i, int j) const { return a[(size_t)i * s + j] != 0; }
};

// Level-synchronous peeling (the definition of core numbers and peel rounds
// used throughout): start at level k = 0; in each sub-round remove every
// remaining vertex whose remaining degree is <= k (all at once), giving them
// core k and the next round number; when nothing is removable, raise k to the
// minimum remaining degree.  Returns the number of rounds.
template <class Nbrs>
int32_t peel_levels(int64_t n, const std::vector<int64_t> &deg0, Nbrs nbrs, int32_t *core,
                    int32_t *round) {
  std::vector<int64_t> deg(deg0);
  std::vector<uint8_t> alive(n, 1);
  std::vector<int64_t> remaining(n);
  for (int64_t v = 0; v < n; v++) remaining[v] = v;
  int64_t k = 0;
  int32_t r = 0;
  std::vector<int64_t> R, next;
  for (int64_t v = 0; v < n; v++)
    if (deg[v] <= k) R.push_back(v);
  int64_t left = n;
  while (left > 0) {
    if (R.empty()) {
      // nothing removable at level k: jump to the minimum remaining degree
      std::vector<int64_t> keep;
      int64_t kmin = INT64_MAX;
      for (int64_t v : remaining)
        if (alive[v]) {
          keep.push_back(v);
          kmin = std::min(kmin, deg[v]);
        }
      remaining.swap(keep);
      k = kmin;
      for (int64_t v : remaining)
        if (deg[v] <= k) R.push_back(v);
    }
    for (int64_t v : R) {
      alive[v] = 0;
      core[v] = (int32_t)k;
      round[v] = r;
    }
    left -= (int64_t)R.size();
    next.clear();
    for (int64_t v : R)
      nbrs(v, [&](int64_t u) {
        if (alive[u]) {
          deg[u]--;
          if (deg[u] == k) next.push_back(u);  // crossed from k+1 to k: removable next round
        }
      });
    R.swap(next);
    r++;
  }
  return r;
}

// Greedy colouring (Sec. 3): visit the vertices in the given order and give
// each the smallest positive colour not used by an already coloured neighbour.
// Returns the number of colours L.
int greedy_colour(const Local &G, const std::vector<int> &order, std::vector<int> &colour) {
  colour.assign(G.s, 0);
  int L = 0;
  std::vector<uint8_t> used;
  for (int x : order) {
    used.assign(order.size() + 2, 0);
    for (int y : order)
      if (colour[y] > 0 && G.adj(x, y)) used[colour[y]] = 1;
    int c = 1;
    while (used[c]) c++;
    colour[x] = c;
    L = std::max(L, c);
  }
  return L;
}

Local induced(const Csr &g, const std::vector<int32_t> &vs) {
  Local G;
  G.s = (int)vs.size();
  G.a.assign((size_t)G.s * G.s, 0);
  for (int i = 0; i < G.s; i++)
    for (int j = i + 1; j < G.s; j++)
      if (adjacent(g, vs[i], vs[j])) G.a[(size_t)i * G.s + j] = G.a[(size_t)j * G.s + i] = 1;
  return G;
}

void local_peel(const Local &G, const std::vector<int> &members, std::vector<int32_t> &kn,
                std::vector<int32_t> &lround) {
  // peel the subgraph induced by `members` (indices into G)
  int64_t s = (int64_t)members.size();
  std::vector<int64_t> deg(s, 0);
  for (int64_t i = 0; i < s; i++)
    for (int64_t j = 0; j < s; j++)
      if (i != j && G.adj(members[i], members[j])) deg[i]++;
  std::vector<int32_t> c(s), r(s);
  peel_levels(s, deg,
              [&](int64_t i, auto &&f) {
                for (int64_t j = 0; j < s; j++)
                  if (j != i && G.adj(members[i], members[j])) f(j);
              },
              c.data(), r.data());
  kn.assign(G.s, -1);
  lround.assign(G.s, -1);
  for (int64_t i = 0; i < s; i++) {
    kn[members[i]] = c[i];
    lround[members[i]] = r[i];
  }
}

struct Stats {
  int64_t kmax = 0, nrounds = 0, heuristic = 0, omega = 0, certified_early = 0;
  int64_t survivors = 0, roots_visited = 0, roots_branched = 0, nodes = 0;
  int64_t pruned_size = 0, pruned_kn = 0, pruned_colour = 0;
};

// State shared by the workers of the threaded search (Sec. 4.5: workers take
// vertices from a task queue and tell each other every improved bound; here
// the bound is one atomic word read before every bound test and the best
// clique is updated under a lock).
struct Shared {
  std::atomic<int64_t> bound{0};
  std::mutex mu;
  std::vector<int32_t> H;
};

void raise_to(std::atomic<int64_t> &a, int64_t v) {
  int64_t cur = a.load(std::memory_order_relaxed);
  while (cur < v && !a.compare_exchange_weak(cur, v, std::memory_order_relaxed)) {
  }
}

struct Solver {
  Csr g;
  const int32_t *core = nullptr;  // K(v)
  const int32_t *rank = nullptr;  // degeneracy rank (position in the search order)
  bool native = false;            // search order = vertex id (the "native" variant)
  std::vector<int32_t> H;         // best clique (original ids)
  int64_t hsize = 0;              // |H| (may be a phantom bound in frozen mode)
  Stats st;
  bool use_neigh_cores = true;
  Shared *sh = nullptr;           // threaded mode: the shared bound and clique

  // Position of v in the order the roots are searched in; a root's reduced
  // neighbourhood holds only its neighbours that come later.
  int64_t key(int32_t v) const { return native ? (int64_t)v : (int64_t)rank[v]; }

  // The current bound |H|: in threaded mode every worker's improvements count.
  int64_t bound() {
    if (sh) hsize = std::max(hsize, sh->bound.load(std::memory_order_relaxed));
    return hsize;
  }

  // A clique larger than the bound was found.
  void publish(const std::vector<int32_t> &ids) {
    if (!sh) {
      H = ids;
      hsize = (int64_t)H.size();
      return;
    }
    std::lock_guard<std::mutex> lk(sh->mu);
    if ((int64_t)ids.size() > sh->bound.load(std::memory_order_relaxed)) {
      sh->H = ids;
      sh->bound.store((int64_t)ids.size(), std::memory_order_relaxed);
    }
    hsize = std::max(hsize, sh->bound.load(std::memory_order_relaxed));
  }

  // Branch(C, P) of Alg. 2.  P holds (local index, colour) in colouring
  // order; `ids` maps local indices to original vertex ids.
  void branch(const Local &G, const std::vector<int32_t> &ids, std::vector<int32_t> &C,
              std::vector<std::pair<int, int>> P) {
    st.nodes++;
    while (!P.empty() && (int64_t)(P.size() + C.size()) > bound()) {
      // R8: the largest colour, ties to the latest in colouring order
      size_t pick = 0;
      for (size_t t = 0; t < P.size(); t++)
        if (P[t].second >= P[pick].second) pick = t;
      int u = P[pick].first;
      P.erase(P.begin() + (long)pick);
      C.push_back(u);
      // P' = P intersect N_R(u): neighbours of u still in P and not removed by
      // the core bound against the current |H| (implicit removal after a new clique, Alg. 2)
      std::vector<int> Pn;
      for (auto &e : P)
        if (G.adj(u, e.first) && core[ids[e.first]] >= hsize) Pn.push_back(e.first);
      if (!Pn.empty()) {
        std::sort(Pn.begin(), Pn.end());  // R7: natural order = increasing local index
        std::vector<int> colour;
        int L = greedy_colour(G, Pn, colour);
        if ((int64_t)C.size() + L > hsize) {
          std::vector<std::pair<int, int>> Pc;
          for (int x : Pn) Pc.push_back({x, colour[x]});
          branch(G, ids, C, Pc);
        }
      } else if ((int64_t)C.size() > hsize) {
        std::vector<int32_t> found;
        for (int x : C) found.push_back(ids[x]);
        publish(found);
      }
      C.pop_back();
    }
  }

  // InitialBranch(v) of Alg. 2 on the closed reduced neighbourhood N_R(v).
  // Fills the optional per-root report (open-neighbourhood quantities).
  void initial_branch(int32_t v, int32_t *rep) {
    st.roots_visited++;
    const int64_t b0 = bound();
    std::vector<int32_t> P{v};
    for (int64_t e = g.off[v]; e < g.off[v + 1]; e++) {
      int32_t u = g.idx[e];
      if (key(u) > key(v) && core[u] >= b0) P.push_back(u);
    }
    std::sort(P.begin() + 1, P.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });
    if (rep) rep[0] = (int32_t)P.size() - 1;
    if ((int64_t)P.size() <= bound()) { st.pruned_size++; return; }  // size test
    Local G = induced(g, P);
    std::vector<int> all(G.s);
    for (int i = 0; i < G.s; i++) all[i] = i;
    std::vector<int32_t> kn, lround;
    local_peel(G, all, kn, lround);  // neighbourhood core numbers K_N
    int32_t KP = *std::max_element(kn.begin(), kn.end());  // K(P)
    if (rep) rep[1] = KP - 1;
    const int64_t b1 = bound();
    if (use_neigh_cores && KP < b1) { st.pruned_kn++; return; }  // core test (R4)
    std::vector<int> keep;  // drop K_N(x) < |H|
    for (int i = 0; i < G.s; i++)
      if (!use_neigh_cores || kn[i] >= b1) keep.push_back(i);
    // (R6) colour in reverse local peel order, i.e. by decreasing
    // (round, index) of the peel of the neighbourhood graph
    std::vector<int> ord(keep);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) {
      if (lround[a] != lround[b]) return lround[a] > lround[b];
      return a > b;
    });
    std::vector<int> colour;
    int L = greedy_colour(G, ord, colour);
    if (rep) rep[2] = L - 1;
    if (L <= bound()) { st.pruned_colour++; return; }  // colouring test
    st.roots_branched++;
    std::vector<std::pair<int, int>> Pc;
    for (int x : ord) Pc.push_back({x, colour[x]});
    std::vector<int32_t> C;
    branch(G, P, C, Pc);
  }
};

// Per-vertex arrays of the peel and the order, owned once and shared
// read-only by every worker.
struct Prep {
  std::vector<int32_t> core, round, rank, order;
  int32_t kmax = 0;
  int32_t nrounds = 0;
};

void prepare(const Csr &g, Prep &p) {
  p.core.resize(g.n);
  p.round.resize(g.n);
  p.rank.resize(g.n);
  p.order.resize(g.n);
  p.nrounds = or_peel(g.n, g.off, g.idx, p.core.data(), p.round.data(), &p.kmax);
  or_rank(g.n, p.round.data(), p.rank.data(), p.order.data());
}

}  // namespace

extern "C" {

// Validate the graph contract: offsets nondecreasing from 0, ids in range,
// rows strictly increasing (sorted, no duplicates), no self-loops, symmetric.
// Returns 0 when valid, else 1 offsets, 2 range, 3 self-loop, 4 order, 5 asymmetric.
int or_validate(int64_t n, const int64_t *off, const int32_t *idx) {
  if (n < 0 || off[0] != 0) return 1;
  for (int64_t v = 0; v < n; v++)
    if (off[v + 1] < off[v]) return 1;
  Csr g{n, off, idx};
  for (int64_t v = 0; v < n; v++)
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      int32_t u = idx[e];
      if (u < 0 || u >= n) return 2;
      if (u == v) return 3;
      if (e > off[v] && idx[e - 1] >= u) return 4;
    }
  for (int64_t v = 0; v < n; v++)
    for (int64_t e = off[v]; e < off[v + 1]; e++)
      if (!adjacent(g, idx[e], (int32_t)v)) return 5;
  return 0;
}

// Core numbers by the bucket algorithm of Batagelj and Zaversnik (cited in
// Sec. 3): process vertices in nondecreasing current degree; each processed
// vertex v fixes K(v) = its current degree and lowers by one the degree of
// every neighbour whose degree is still larger, moving it one bucket down.
void or_core_bz(int64_t n, const int64_t *off, const int32_t *idx, int32_t *core) {
  if (n == 0) return;
  std::vector<int64_t> deg(n), pos(n), vert(n);
  int64_t md = 0;
  for (int64_t v = 0; v < n; v++) {
    deg[v] = off[v + 1] - off[v];
    md = std::max(md, deg[v]);
  }
  std::vector<int64_t> bin(md + 2, 0);
  for (int64_t v = 0; v < n; v++) bin[deg[v]]++;
  int64_t start = 0;
  for (int64_t d = 0; d <= md; d++) {
    int64_t c = bin[d];
    bin[d] = start;
    start += c;
  }
  for (int64_t v = 0; v < n; v++) {
    pos[v] = bin[deg[v]];
    vert[pos[v]] = v;
    bin[deg[v]]++;
  }
  for (int64_t d = md; d >= 1; d--) bin[d] = bin[d - 1];
  bin[0] = 0;
  for (int64_t i = 0; i < n; i++) {
    int64_t v = vert[i];
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
      int64_t u = idx[e];
      if (deg[u] > deg[v]) {
        int64_t du = deg[u], pu = pos[u], pw = bin[du], w = vert[pw];
        if (u != w) {
          pos[u] = pw; vert[pu] = w;
          pos[w] = pu; vert[pw] = u;
        }
        bin[du]++;
        deg[u]--;
      }
    }
  }
  for (int64_t v = 0; v < n; v++) core[v] = (int32_t)deg[v];
}

// Level-synchronous peel of the whole graph: core numbers, peel rounds and the
// largest core number.  Returns the number of rounds.
int32_t or_peel(int64_t n, const int64_t *off, const int32_t *idx, int32_t *core, int32_t *round,
                int32_t *kmax) {
  std::vector<int64_t> deg(n);
  for (int64_t v = 0; v < n; v++) deg[v] = off[v + 1] - off[v];
  int32_t r = peel_levels(n, deg,
                          [&](int64_t v, auto &&f) {
                            for (int64_t e = off[v]; e < off[v + 1]; e++) f(idx[e]);
                          },
                          core, round);
  int32_t km = 0;
  for (int64_t v = 0; v < n; v++) km = std::max(km, core[v]);
  *kmax = km;
  return r;
}

// Degeneracy rank: position of v in increasing (round, id) order; order is the
// inverse permutation.  Counting sort on the round, stable in id.
void or_rank(int64_t n, const int32_t *round, int32_t *rank, int32_t *order) {
  int32_t R = 0;
  for (int64_t v = 0; v < n; v++) R = std::max(R, round[v] + 1);
  std::vector<int64_t> start(R + 1, 0);
  for (int64_t v = 0; v < n; v++) start[round[v] + 1]++;
  for (int32_t r = 0; r < R; r++) start[r + 1] += start[r];
  for (int64_t v = 0; v < n; v++) {
    int64_t p = start[round[v]]++;
    rank[v] = (int32_t)p;
    order[p] = (int32_t)v;
  }
}

// One seed of HeuristicClique (Alg. 1) with readings R1, R2: C = {v}, then
// every neighbour u with K(u) >= tau, by decreasing core order (decreasing
// rank), joins C when it is adjacent to every member of C.
std::vector<int32_t> seed_clique(const Csr &g, int32_t v, int64_t tau, const int32_t *core,
                                 const int32_t *rank) {
  std::vector<int32_t> S;  // neighbours with core >= tau
  for (int64_t e = g.off[v]; e < g.off[v + 1]; e++)
    if (core[g.idx[e]] >= tau) S.push_back(g.idx[e]);
  std::sort(S.begin(), S.end(), [&](int32_t a, int32_t b) { return rank[a] > rank[b]; });
  std::vector<int32_t> C{v};  // (R1)
  for (int32_t u : S) {  // by decreasing core order (R2)
    bool ok = true;  // is C + {u} a clique?
    for (int32_t c : C)
      if (!adjacent(g, u, c)) { ok = false; break; }
    if (ok) C.push_back(u);
  }
  return C;
}

// HeuristicClique (Alg. 1) with readings R1, R2.  frozen_tau < 0: the paper's
// procedure (seeds skipped when K(v) < max; S filtered by K(u) >= max, the
// running maximum).  frozen_tau >= 0: every seed is processed and S is
// filtered by the fixed tau (a deterministic per-seed variant used to compare
// per-seed cliques).  Writes H sorted ascending; returns |H|.
int32_t or_heuristic(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *core,
                     const int32_t *rank, const int32_t *order, int32_t frozen_tau,
                     int32_t *clique) {
  Csr g{n, off, idx};
  std::vector<int32_t> H;
  int64_t mx = 0;
  for (int64_t r = n - 1; r >= 0; r--) {  // seeds by decreasing core order (R2)
    int32_t v = order[r];
    int64_t tau = frozen_tau >= 0 ? frozen_tau : mx;
    if (frozen_tau < 0 && core[v] < mx) continue;  // seed skip test
    std::vector<int32_t> C = seed_clique(g, v, tau, core, rank);
    if ((int64_t)C.size() > mx) {  // strictly larger: new H
      H = C;
      mx = (int64_t)C.size();
    }
  }
  std::sort(H.begin(), H.end());
  for (size_t i = 0; i < H.size(); i++) clique[i] = H[i];
  return (int32_t)H.size();
}

// Clique-peeling vertex order for compression (Sec. 6.2): repeatedly take
// large cliques found by the heuristic, place their vertices next to each
// other, remove them, and continue on what is left.  Reading (the paper runs
// its heuristic and removes one clique per pass): every remaining vertex v
// grows its greedy clique H(v) = {v} + first-fit over its remaining
// neighbours in decreasing degeneracy rank (Alg. 1 with C = {v}); key(v) =
// (|H(v)|, rank(v)); in one pass every clique whose key is the largest among
// the cliques sharing any of its vertices is taken (so the largest clique of
// the pass always is, and taken cliques are disjoint); taken cliques are
// placed by decreasing key, the vertices of a clique by decreasing degree
// (ties by id).  order[p] = vertex at position p, block[b] = first position of
// clique b (block[nb] = n).  Returns nb.
int64_t or_clique_order(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *rank,
                        int32_t *order, int64_t *block) {
  Csr g{n, off, idx};
  std::vector<uint8_t> alive(n, 1);
  std::vector<uint64_t> owner(n);
  int64_t placed = 0, nb = 0;
  auto grow = [&](int32_t v) {
    std::vector<int32_t> S;
    for (int64_t e = off[v]; e < off[v + 1]; e++)
      if (alive[idx[e]]) S.push_back(idx[e]);
    std::sort(S.begin(), S.end(), [&](int32_t a, int32_t b) { return rank[a] > rank[b]; });
    std::vector<int32_t> C{v};
    for (int32_t u : S) {
      bool ok = true;
      for (size_t i = 1; i < C.size() && ok; i++) ok = adjacent(g, u, C[i]);
      if (ok) C.push_back(u);
    }
    return C;
  };
  while (placed < n) {
    std::fill(owner.begin(), owner.end(), 0);
    for (int64_t v = 0; v < n; v++) {
      if (!alive[v]) continue;
      std::vector<int32_t> C = grow((int32_t)v);
      uint64_t key = ((uint64_t)C.size() << 32) | (uint32_t)rank[v];
      for (int32_t x : C) owner[x] = std::max(owner[x], key);
    }
    std::vector<std::pair<uint64_t, std::vector<int32_t>>> taken;
    for (int64_t v = 0; v < n; v++) {
      if (!alive[v]) continue;
      std::vector<int32_t> C = grow((int32_t)v);
      uint64_t key = ((uint64_t)C.size() << 32) | (uint32_t)rank[v];
      bool own = true;
      for (int32_t x : C) own = own && owner[x] == key;
      if (own) taken.push_back({key, C});
    }
    std::sort(taken.begin(), taken.end(),
              [](const auto &a, const auto &b) { return a.first > b.first; });
    for (auto &t : taken) {
      std::vector<int32_t> C = t.second;
      std::sort(C.begin(), C.end(), [&](int32_t a, int32_t b) {
        return g.deg(a) != g.deg(b) ? g.deg(a) > g.deg(b) : a < b;
      });
      block[nb++] = placed;
      for (int32_t x : C) {
        order[placed++] = x;
        alive[x] = 0;
      }
    }
  }
  block[nb] = n;
  return nb;
}

// Strong-reachability graph of a temporal network (Sec. 6.1).  Temporal edges
// (src[e] -> dst[e]) are given in time order; a temporal path uses edges in
// increasing position of that order (the paper's increasing edge times; with
// equal times the input order decides).  R[x] = {x} plus every vertex with a
// temporal path to x, built by sweeping the edges in order (R[dst] gets R[src]).
// {a, b} is an edge of the result iff a reaches b and b reaches a (a != b).
// Writes the CSR (rows sorted) into off[n+1] / adj[capacity]; returns the
// number of entries (also when it exceeds capacity, then nothing past it).
int64_t or_strong_reach(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                        int64_t *off, int32_t *adj, int64_t capacity) {
  const int64_t W = (n + 63) / 64;
  std::vector<uint64_t> R((size_t)(n * W), 0);
  for (int64_t x = 0; x < n; x++) R[(size_t)(x * W + x / 64)] |= 1ull << (x % 64);
  for (int64_t e = 0; e < m; e++) {
    const int64_t u = src[e], v = dst[e];
    for (int64_t w = 0; w < W; w++) R[(size_t)(v * W + w)] |= R[(size_t)(u * W + w)];
  }
  auto reaches = [&](int64_t a, int64_t b) {  // a has a temporal path to b
    return (R[(size_t)(b * W + a / 64)] >> (a % 64)) & 1ull;
  };
  int64_t k = 0;
  off[0] = 0;
  for (int64_t x = 0; x < n; x++) {
    for (int64_t s = 0; s < n; s++)
      if (s != x && reaches(s, x) && reaches(x, s)) {
        if (k < capacity) adj[k] = (int32_t)s;
        k++;
      }
    off[x + 1] = k;
  }
  return k;
}

// First rank whose core number is >= bound (ranks are nondecreasing in core).
int32_t or_r0(int64_t n, const int32_t *core, const int32_t *order, int32_t bound) {
  int64_t r = 0;
  while (r < n && core[order[r]] < bound) r++;
  return (int32_t)r;
}

// Explicit pruning (Alg. 2, after the heuristic) and orientation: for every vertex of rank >=
// r0 (core >= bound) the list of its higher-ranked neighbours, relabelled to
// rank - r0 and sorted.  poff has n - r0 + 1 entries.  Returns r0.
int32_t or_prune_orient(int64_t n, const int64_t *off, const int32_t *idx, const int32_t *core,
                        const int32_t *rank, const int32_t *order, int32_t bound, int64_t *poff,
                        int32_t *padj) {
  int32_t r0 = or_r0(n, core, order, bound);
  int64_t w = 0;
  poff[0] = 0;
  for (int64_t r = r0; r < n; r++) {
    int32_t v = order[r];
    int64_t b = w;
    for (int64_t e = off[v]; e < off[v + 1]; e++)
      if (rank[idx[e]] > rank[v]) padj[w++] = rank[idx[e]] - r0;
    std::sort(padj + b, padj + w);
    poff[r - r0 + 1] = w;
  }
  return r0;
}

// MaxClique (Alg. 2), with the variants and test modes of the paper's
// experiments.  stats (optional, 13 int64): kmax, nrounds, heuristic size,
// omega, certified by Fact 1 after the heuristic, survivors of the initial
// pruning, roots visited, roots branched, Branch calls, roots pruned by the
// size test, by the neighbourhood-core test, by the colouring test, and the
// size of the returned clique.
//   use_neigh_cores = 0: the "no neighbourhood cores" variant (Sec. 5).
//   native = 1: roots are searched in vertex-id order and each root's reduced
//     neighbourhood holds its neighbours of larger id (the "native order"
//     variant of Sec. 5); 0: degeneracy order (the method, R3).
//   threads = T > 1: the parallel search of Sec. 4.5 -- the heuristic's seeds
//     and then the roots are taken from a shared counter by T workers, every
//     bound test reads the shared bound, and an improved clique replaces the
//     best one under a lock.  The result is omega whatever the interleaving;
//     which maximum clique is returned, and the heuristic's size, may vary.
//   dispatch (NULL or a permutation of the vertices): the order in which the
//     roots are taken; every root still searches only its reduced
//     neighbourhood in the search order, so the result is unchanged.
//   inject_at / inject_val (ninject pairs, inject_at nondecreasing): before
//     the root at dispatch position inject_at[i] starts, the bound is raised to
//     inject_val[i] with no clique behind it, as if another worker had found
//     one (the scripted stand-in for racing workers).  With injected values
//     below omega the returned clique is still a maximum clique.
// Returns the final bound (omega, or an injected value if larger); writes the
// best clique found, sorted ascending, into clique (capacity >= kmax + 1).
int32_t or_max_clique_ex(int64_t n, const int64_t *off, const int32_t *idx,
                         int32_t use_neigh_cores, int32_t native, int32_t threads,
                         const int32_t *dispatch, int64_t ninject, const int64_t *inject_at,
                         const int32_t *inject_val, int32_t *clique, int64_t *stats) {
  if (n == 0) {
    if (stats) std::memset(stats, 0, 13 * sizeof(int64_t));
    return 0;
  }
  const Csr g{n, off, idx};
  const int T = std::max(1, (int)threads);
  Prep p;
  prepare(g, p);  // CoreNumbers and the degeneracy order
  Stats tot;
  tot.kmax = p.kmax;
  tot.nrounds = p.nrounds;
  Shared sh;
  // HeuristicClique: T workers over the seeds by decreasing core order,
  // sharing the running maximum (T = 1: Alg. 1 exactly)
  {
    std::atomic<int64_t> next{0};
    auto work = [&]() {
      for (;;) {
        const int64_t i = next.fetch_add(1);
        if (i >= n) break;
        const int32_t v = p.order[n - 1 - i];
        const int64_t mx = sh.bound.load(std::memory_order_relaxed);
        if (p.core[v] < mx) continue;  // seed skip test
        std::vector<int32_t> C = seed_clique(g, v, mx, p.core.data(), p.rank.data());
        if ((int64_t)C.size() > sh.bound.load(std::memory_order_relaxed)) {
          std::lock_guard<std::mutex> lk(sh.mu);
          if ((int64_t)C.size() > sh.bound.load(std::memory_order_relaxed)) {
            sh.H = C;
            sh.bound.store((int64_t)C.size(), std::memory_order_relaxed);
          }
        }
      }
    };
    if (T == 1) {
      work();
    } else {
      std::vector<std::thread> ws;
      for (int t = 0; t < T; t++) ws.emplace_back(work);
      for (auto &w : ws) w.join();
    }
  }
  const int64_t h = sh.bound.load();
  tot.heuristic = h;
  if (h == p.kmax + 1) {
    tot.certified_early = 1;  // Fact 1: nothing larger can exist
  } else {
    for (int64_t v = 0; v < n; v++) tot.survivors += p.core[v] >= h;  // explicit removal of K(v) < |H|
    std::vector<int32_t> seq(n);
    for (int64_t i = 0; i < n; i++)
      seq[i] = dispatch ? dispatch[i] : native ? (int32_t)i : p.order[i];
    std::atomic<int64_t> next{0};
    std::vector<Stats> part(T);
    auto work = [&](int t) {
      Solver S;
      S.g = g;
      S.core = p.core.data();
      S.rank = p.rank.data();
      S.native = native != 0;
      S.use_neigh_cores = use_neigh_cores != 0;
      S.sh = &sh;
      for (;;) {  // main loop: take the next root from the queue
        const int64_t i = next.fetch_add(1);
        if (i >= n) break;
        for (int64_t k = 0; k < ninject; k++)
          if (inject_at[k] == i) raise_to(sh.bound, inject_val[k]);
        const int32_t v = seq[i];
        if (p.core[v] < S.bound()) continue;  // removed explicitly or implicitly
        S.initial_branch(v, nullptr);
      }
      part[t] = S.st;
    };
    if (T == 1) {
      work(0);
    } else {
      std::vector<std::thread> ws;
      for (int t = 0; t < T; t++) ws.emplace_back(work, t);
      for (auto &w : ws) w.join();
    }
    for (const Stats &q : part) {
      tot.roots_visited += q.roots_visited;
      tot.roots_branched += q.roots_branched;
      tot.nodes += q.nodes;
      tot.pruned_size += q.pruned_size;
      tot.pruned_kn += q.pruned_kn;
      tot.pruned_colour += q.pruned_colour;
    }
  }
  std::vector<int32_t> H = sh.H;
  std::sort(H.begin(), H.end());
  for (size_t i = 0; i < H.size(); i++) clique[i] = H[i];
  tot.omega = sh.bound.load();
  if (stats) {
    int64_t v[13] = {tot.kmax,          tot.nrounds,       tot.heuristic,
                     tot.omega,         tot.certified_early, tot.survivors,
                     tot.roots_visited, tot.roots_branched,  tot.nodes,
                     tot.pruned_size,   tot.pruned_kn,       tot.pruned_colour,
                     (int64_t)H.size()};
    std::memcpy(stats, v, sizeof(v));
  }
  return (int32_t)tot.omega;
}

// MaxClique (Alg. 2), serial, degeneracy order: or_max_clique_ex with one
// worker and no injections.  stats (optional) takes the first 12 values.
int32_t or_max_clique(int64_t n, const int64_t *off, const int32_t *idx, int32_t use_neigh_cores,
                      int32_t *clique, int64_t *stats) {
  int64_t st[13];
  int32_t w = or_max_clique_ex(n, off, idx, use_neigh_cores, 0, 1, nullptr, 0, nullptr, nullptr,
                               clique, st);
  if (stats) std::memcpy(stats, st, 12 * sizeof(int64_t));
  return w;
}

// Per-root search with a frozen bound b and no sharing between roots: for
// every vertex v with K(v) >= b, InitialBranch(v) runs with a phantom clique
// of size b.  Outputs (indexed by vertex id, -1 when not reached):
//   s_out:    |N+(v)| restricted to K >= b (the open neighbourhood size)
//   kn_out:   largest core number of the open neighbourhood graph
//   l_out:    colours used by the open neighbourhood in reverse peel order
//   omega_out: 1 + omega(G[N+(v)]) when that exceeds b, else 0.
// (Open-neighbourhood values are the closed ones minus one: the root is
// adjacent to every vertex of its neighbourhood.)  native = 1: the
// neighbourhoods are oriented by vertex id, as in or_max_clique_ex.
void or_root_omega_ex(int64_t n, const int64_t *off, const int32_t *idx, int32_t b,
                      int32_t native, int32_t *s_out, int32_t *kn_out, int32_t *l_out,
                      int32_t *omega_out) {
  const Csr g{n, off, idx};
  Prep p;
  prepare(g, p);
  Solver S;
  S.g = g;
  S.core = p.core.data();
  S.rank = p.rank.data();
  S.native = native != 0;
  for (int64_t v = 0; v < n; v++) s_out[v] = kn_out[v] = l_out[v] = omega_out[v] = -1;
  for (int64_t v = 0; v < n; v++) {
    if (p.core[v] < b) continue;
    S.hsize = b;
    S.H.clear();
    int32_t rep[3] = {-1, -1, -1};
    S.initial_branch((int32_t)v, rep);
    s_out[v] = rep[0];
    kn_out[v] = rep[1];
    l_out[v] = rep[2];
    omega_out[v] = S.hsize > b ? (int32_t)S.hsize : 0;
  }
}

void or_root_omega(int64_t n, const int64_t *off, const int32_t *idx, int32_t b, int32_t *s_out,
                   int32_t *kn_out, int32_t *l_out, int32_t *omega_out) {
  or_root_omega_ex(n, off, idx, b, 0, s_out, kn_out, l_out, omega_out);
}

// Utilities on an explicit small graph (dense 0/1 matrix, s x s), exposed so
// the tests can check them directly.
void or_local_peel(int32_t s, const uint8_t *adj, int32_t *kn, int32_t *lround) {
  Local G;
  G.s = s;
  G.a.assign(adj, adj + (size_t)s * s);
  std::vector<int> all(s);
  for (int i = 0; i < s; i++) all[i] = i;
  std::vector<int32_t> k, r;
  local_peel(G, all, k, r);
  for (int i = 0; i < s; i++) { kn[i] = k[i]; lround[i] = r[i]; }
}

int32_t or_greedy_colour(int32_t s, const uint8_t *adj, const int32_t *order, int32_t len,
                         int32_t *colour) {
  Local G;
  G.s = s;
  G.a.assign(adj, adj + (size_t)s * s);
  std::vector<int> ord(order, order + len), col;
  int L = greedy_colour(G, ord, col);
  for (int i = 0; i < s; i++) colour[i] = col[i];
  return L;
}

}  // extern "C"
