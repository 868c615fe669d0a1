// Host side of the single-pass HBM kernel: the order in which its wavefronts walk
// the qubits, and the gather words along it.  A qubit reads the other stored words of
// each of its checks, which the check's other qubits read too; the re-reads are
// served by L2 only while the check's qubits sit close together in the walk.
// Candidates: breadth-first levels from a pseudo-peripheral qubit (the end of a
// repeated farthest-first search; neighbours = qubits sharing a check, taken by
// increasing degree) cut a lattice into thin slices; groups of B consecutive levels
// form bands, and each band is walked breadth first along its length from a
// pseudo-peripheral qubit of the band (B = 0 walks the levels themselves:
// Cuthill-McKee); the band width with the fewest misses in a model of one
// workgroup's share of L2 is kept.  Given qubit coordinates, strips of k consecutive
// coordinate values walked row by row are candidates too; the best of them replaces
// the band walk only if the model gives it at most 0.9 of the band walk's misses
// (measured: planar d=31's strips, 1 % fewer modelled misses, ran 1 % slower; toric
// L=32's, 19 % fewer, cut the HBM reads by 6 % and the time by 1 %).
#include <algorithm>
#include <cstdint>
#include <vector>

#include "bp4_gather.h"

namespace bp4 {
namespace {

struct WalkGraph {
    int n = 0, m = 0;
    std::vector<std::vector<int32_t>> adj;     // neighbours by increasing degree
    std::vector<std::vector<int32_t>> vchecks; // checks of each qubit
    std::vector<std::vector<int32_t>> cq;      // qubits of each check, by position
};

// Breadth-first search from s over the qubits with ok[v]; appends the visit order
// to `out` and returns the depth.  lev: scratch, -1 outside the search.
int32_t bfs_order(const WalkGraph &G, int32_t s, const std::vector<uint8_t> &ok, std::vector<int32_t> &lev,
                  std::vector<int32_t> &out)
{
    const size_t b = out.size();
    lev[s] = 0;
    out.push_back(s);
    for (size_t h = b; h < out.size(); ++h) {
        const int32_t v = out[h];
        for (int32_t u : G.adj[v])
            if (ok[u] && lev[u] < 0) {
                lev[u] = lev[v] + 1;
                out.push_back(u);
            }
    }
    return lev[out.back()];
}

// Pseudo-peripheral qubit of s's component among ok[]: repeated farthest-first
// search (up to 8 rounds), ending at a least-degree qubit of the deepest level.
int32_t peripheral(const WalkGraph &G, int32_t s, const std::vector<uint8_t> &ok)
{
    std::vector<int32_t> lev(G.n, -1), q;
    int32_t depth = bfs_order(G, s, ok, lev, q);
    for (int k = 0; k < 8; ++k) {
        int32_t far = q.back();
        for (int32_t v : q)
            if (lev[v] == depth && G.adj[v].size() < G.adj[far].size()) far = v;
        std::vector<int32_t> lev2(G.n, -1), q2;
        const int32_t d2 = bfs_order(G, far, ok, lev2, q2);
        if (d2 <= depth) break;
        s = far;
        depth = d2;
        q.swap(q2);
        lev.swap(lev2);
    }
    return s;
}

// Breadth-first walk of the qubits with ok[] (component by component, each from a
// pseudo-peripheral start of least degree), appended to `order`; lev gets the depth.
void walk_components(const WalkGraph &G, std::vector<uint8_t> ok, std::vector<int32_t> &order,
                     std::vector<int32_t> *lev_out)
{
    std::vector<int32_t> lev(G.n, -1);
    for (;;) {
        int32_t s = -1;
        for (int32_t v = 0; v < G.n; ++v)
            if (ok[v] && (s < 0 || G.adj[v].size() < G.adj[s].size())) s = v;
        if (s < 0) break;
        s = peripheral(G, s, ok);
        const size_t b = order.size();
        bfs_order(G, s, ok, lev, order);
        for (size_t h = b; h < order.size(); ++h) ok[order[h]] = 0;
    }
    if (lev_out) *lev_out = lev;
}

std::vector<int32_t> banded_walk(const WalkGraph &G, int B)
{
    std::vector<int32_t> cm, lev;
    walk_components(G, std::vector<uint8_t>(G.n, 1), cm, &lev);
    if (B <= 0) return cm;
    int32_t maxlev = 0;
    for (int32_t v = 0; v < G.n; ++v) maxlev = std::max(maxlev, lev[v]);
    std::vector<int32_t> order;
    order.reserve(G.n);
    for (int32_t b = 0; b <= maxlev / B; ++b) {
        std::vector<uint8_t> ok(G.n, 0);
        for (int32_t v = 0; v < G.n; ++v) ok[v] = lev[v] / B == b;
        walk_components(G, ok, order, nullptr);
    }
    return order;
}

// Strips of k consecutive values of coordinate `a` (values ranked), walked along
// coordinate `b`, then `a`.
std::vector<int32_t> strip_walk(int n, const int32_t *xy, int a, int k)
{
    std::vector<int32_t> vals(n);
    for (int v = 0; v < n; ++v) vals[v] = xy[2 * v + a];
    std::sort(vals.begin(), vals.end());
    vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
    std::vector<int32_t> strip(n), order(n);
    for (int v = 0; v < n; ++v)
        strip[v] = (int32_t)(std::lower_bound(vals.begin(), vals.end(), xy[2 * v + a]) - vals.begin()) / k;
    for (int v = 0; v < n; ++v) order[v] = v;
    std::stable_sort(order.begin(), order.end(), [&](int32_t u, int32_t v) {
        if (strip[u] != strip[v]) return strip[u] < strip[v];
        if (xy[2 * u + 1 - a] != xy[2 * v + 1 - a]) return xy[2 * u + 1 - a] < xy[2 * v + 1 - a];
        return xy[2 * u + a] < xy[2 * v + a];
    });
    return order;
}

// L2 misses of one pass of one workgroup over the walk, summed over LRU caches of
// 160, 192 and 256 record rows (a workgroup's share of an XCD's L2 is 256 rows of
// 256 bytes; of two band widths of planar d=31 the one with fewer modelled misses at
// these capacities, 8, also read fewer bytes from HBM than 5, which wins at 128).  Per position, in the
// kernel's order: the three other stored words of each of the qubit's checks and its
// three state rows are read from the previous record, its state rows and words are
// written to the next one (writes take cache rows, only reads count as misses).
// Stack distances from a Fenwick tree over access times.
constexpr int kCaps[3] = {160, 192, 256};

long walk_misses(const WalkGraph &G, const std::vector<int32_t> &order)
{
    const int64_t rows = 4 * (int64_t)G.m + 3 * (int64_t)G.n;   // rows of one record
    std::vector<int64_t> last((size_t)(2 * rows), -1);
    std::vector<int32_t> fen;
    int64_t t = 0;
    long miss = 0;
    auto add = [&](int64_t i, int32_t d) {
        for (++i; i <= (int64_t)fen.size(); i += i & -i) fen[(size_t)i - 1] += d;
    };
    auto sum = [&](int64_t i) {   // marks at times < i
        int32_t r = 0;
        for (; i > 0; i -= i & -i) r += fen[(size_t)i - 1];
        return r;
    };
    size_t T = 0;
    for (int32_t v : order) T += G.vchecks[v].size() * 4 + 6;
    fen.assign(T, 0);
    auto touch = [&](int64_t key, bool read) {
        const int64_t l = last[(size_t)key];
        if (l < 0) {
            if (read) miss += 3;
        } else {
            const int32_t d = sum(t) - sum(l + 1);   // distinct rows since the last access
            if (read)
                for (int cap : kCaps) miss += d >= cap ? 1 : 0;
            add(l, -1);
        }
        add(t, 1);
        last[(size_t)key] = t++;
    };
    for (size_t i = 0; i < order.size(); ++i) {
        const int32_t v = order[i];
        for (int32_t c : G.vchecks[v]) {
            int p = 0;
            while (G.cq[c][p] != v) ++p;
            for (int q = 0; q < 4; ++q)
                if (q != p) touch(4 * (int64_t)c + q, true);
        }
        for (int k = 0; k < 3; ++k) touch(4 * (int64_t)G.m + 3 * (int64_t)i + k, true);
        for (int k = 0; k < 3; ++k) touch(rows + 4 * (int64_t)G.m + 3 * (int64_t)i + k, false);
        for (int32_t c : G.vchecks[v]) {
            int p = 0;
            while (G.cq[c][p] != v) ++p;
            touch(rows + 4 * (int64_t)c + p, false);
        }
    }
    return miss;
}

}  // namespace

void build_gather_walk(const GatherWalkInput &in, const int32_t *xy, std::vector<uint32_t> &gord,
                       std::vector<uint32_t> &gedge)
{
    const int n = in.n, m = in.m;
    WalkGraph G;
    G.n = n;
    G.m = m;
    G.cq.assign(m, std::vector<int32_t>());
    for (int c = 0; c < m; ++c)
        for (int k = 0; k < in.cstride; ++k) {
            const uint32_t w = in.cedge[(size_t)c * in.cstride + k];
            if (!edge_is_pad(w)) G.cq[c].push_back((int32_t)edge_var(w));
        }
    G.adj.resize(n);
    G.vchecks.resize(n);
    for (int v = 0; v < n; ++v) {
        for (int32_t s = in.vptr[v]; s < in.vptr[v + 1]; ++s) {
            G.vchecks[v].push_back((int32_t)in.vchk[s]);
            for (int32_t u : G.cq[in.vchk[s]])
                if (u != v) G.adj[v].push_back(u);
        }
        std::sort(G.adj[v].begin(), G.adj[v].end());
        G.adj[v].erase(std::unique(G.adj[v].begin(), G.adj[v].end()), G.adj[v].end());
    }
    for (int v = 0; v < n; ++v)
        std::stable_sort(G.adj[v].begin(), G.adj[v].end(),
                         [&](int32_t a, int32_t b) { return G.adj[a].size() < G.adj[b].size(); });
    std::vector<int32_t> best;
    long best_miss = -1;
    for (int B : {0, 3, 4, 5, 6, 8}) {
        std::vector<int32_t> o = banded_walk(G, B);
        const long f = walk_misses(G, o);
        if (best_miss < 0 || f < best_miss) {
            best_miss = f;
            best.swap(o);
        }
    }
    if (xy) {
        const long bar = best_miss - best_miss / 10;
        for (int a = 0; a < 2; ++a)
            for (int k : {2, 3, 4, 6, 8, 10, 12, 16}) {
                std::vector<int32_t> o = strip_walk(n, xy, a, k);
                const long f = walk_misses(G, o);
                if (f <= bar && f < best_miss) {
                    best_miss = f;
                    best.swap(o);
                }
            }
    }
    gord.assign(best.begin(), best.end());
    gedge.assign((size_t)4 * n, kGatherAbsent);
    for (int i = 0; i < n; ++i) {
        const int v = (int)gord[i];
        for (int32_t s = in.vptr[v]; s < in.vptr[v + 1]; ++s) {
            const uint32_t c = in.vchk[s];
            const uint32_t pad = (0xFu << G.cq[c].size()) & 0xFu;
            gedge[(size_t)4 * i + (s - in.vptr[v])] = (4u * c + (uint32_t)in.cpos[s]) | (pad << 20);
        }
    }
}


}  // namespace bp4
