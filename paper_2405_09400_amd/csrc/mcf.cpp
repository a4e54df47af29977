// Integer min-cost flow on a bipartite transportation graph by the primal network simplex
// method (the host step of the flow update, problem (MinCostFlow) of Sec. 3.1-3.2).
//
// Graph: left nodes 0..n-1 (supply s_i), right nodes n..2n-1 (demand s_j), arcs i -> n+j
// with integer costs and no upper bound.  An artificial root joins every node with an
// arc of cost ART larger than any path of real arcs; the initial tree is strongly feasible
// (zero-flow tree arcs point away from the root) and, where the graph has self arcs, is a
// spanning tree of real arcs carrying the identity flow (see below).  Pricing keeps a
// candidate list of eligible arcs between scans (see the loop); the leaving arc is
// the last blocking arc met when the pivot cycle is walked in its orientation from the
// apex, which keeps the tree strongly feasible and rules out cycling.  After a pivot the
// cut-off subtree is re-rooted at the entering arc; the potentials change by one constant on
// one side of the entering arc, so the smaller side (by the subtree sizes the tree keeps) is
// shifted, by a walk over explicit child lists.  The apex of a pivot cycle is found by
// climbing from both ends in turn, and subtree sizes change only below it, so the tree
// bookkeeping of a pivot costs the length of its cycle, not the depth of the tree.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "mcf.hpp"

namespace dd {

struct Simplex {
    int V = 0, M = 0, R = 0;  // nodes (incl. root), real arcs, root id
    std::vector<int> src, dst;
    std::vector<int64_t> cost, flow;
    std::vector<int8_t> state;  // 0 tree, 1 at lower bound
    std::vector<int> parent, pred, size, first_child, next_sib, prev_sib, mark;
    std::vector<int64_t> pot;
    int stamp = 0;

    int64_t rc(int a) const { return cost[a] + pot[src[a]] - pot[dst[a]]; }

    void link_child(int p, int c) {
        parent[c] = p;
        prev_sib[c] = -1;
        next_sib[c] = first_child[p];
        if (first_child[p] >= 0) prev_sib[first_child[p]] = c;
        first_child[p] = c;
    }
    void unlink_child(int c) {
        const int p = parent[c];
        if (prev_sib[c] >= 0)
            next_sib[prev_sib[c]] = next_sib[c];
        else
            first_child[p] = next_sib[c];
        if (next_sib[c] >= 0) prev_sib[next_sib[c]] = prev_sib[c];
        prev_sib[c] = next_sib[c] = -1;
    }

    // nearest common ancestor of a and b: the two ends climb in turn, each marking what it
    // passes, until one reaches a node the other has marked, so the cost is the length of
    // the pivot cycle rather than the depth of the tree
    int apex(int a, int b) {
        if (a == b) return a;
        if (stamp > (1 << 30)) {  // a long run of warm-started solves: restart the stamps
            std::fill(mark.begin(), mark.end(), 0);
            stamp = 0;
        }
        stamp += 2;
        const int ma = stamp - 1, mb = stamp;
        mark[a] = ma;
        mark[b] = mb;
        for (;;) {
            if (parent[a] >= 0) {
                a = parent[a];
                if (mark[a] == mb) return a;
                mark[a] = ma;
            }
            if (parent[b] >= 0) {
                b = parent[b];
                if (mark[b] == ma) return b;
                mark[b] = mb;
            }
        }
    }

    // add d to the potentials of the subtree rooted at r (skip < 0), or of the whole tree
    // except the subtree rooted at skip (r = the root)
    void shift(int r, int skip, int64_t d, std::vector<int>& stack) {
        stack.clear();
        stack.push_back(r);
        while (!stack.empty()) {
            const int x = stack.back();
            stack.pop_back();
            pot[x] += d;
            for (int c = first_child[x]; c >= 0; c = next_sib[c])
                if (c != skip) stack.push_back(c);
        }
    }
};

// A solved problem kept for the next one on the same graph and supplies (the flow update of
// successive B iterations): its optimal basis is a strongly feasible start for new costs.
struct McfWarm {
    bool valid = false;
    int n = 0, m = 0;
    std::vector<int32_t> tail, head;
    std::vector<int64_t> supply;
    Simplex S;
};

McfWarm* mcf_warm_create() { return new McfWarm(); }
void mcf_warm_free(McfWarm* w) { delete w; }

int mcf_network_simplex(int n, int m, const int32_t* tail, const int32_t* head,
                        const int64_t* cost, const int64_t* supply, int64_t* flow_out,
                        int64_t* pot_out) {
    return mcf_network_simplex_warm(n, m, tail, head, cost, supply, flow_out, pot_out, nullptr);
}

int mcf_network_simplex_warm(int n, int m, const int32_t* tail, const int32_t* head,
                             const int64_t* cost, const int64_t* supply, int64_t* flow_out,
                             int64_t* pot_out, McfWarm* warm) {
    const bool reuse = warm && warm->valid && warm->n == n && warm->m == m &&
                       std::equal(tail, tail + m, warm->tail.begin()) &&
                       std::equal(head, head + m, warm->head.begin()) &&
                       std::equal(supply, supply + n, warm->supply.begin());
    Simplex fresh;
    Simplex& S = reuse ? warm->S : fresh;
    if (warm) warm->valid = false;  // until this solve ends
    const int N2 = 2 * n;
    S.V = N2 + 1;
    S.R = N2;
    S.M = m;
    const int A = m + N2;  // real + artificial arcs
    S.src.resize(A);
    S.dst.resize(A);
    S.cost.resize(A);
    if (!reuse) {
        S.flow.assign(A, 0);
        S.state.assign(A, 1);
    }
    int64_t maxc = 1, tot = 0;
    for (int a = 0; a < m; ++a) {
        if (tail[a] < 0 || tail[a] >= n || head[a] < 0 || head[a] >= n) return -2;
        S.src[a] = tail[a];
        S.dst[a] = n + head[a];
        S.cost[a] = cost[a];
        maxc = std::max<int64_t>(maxc, std::llabs(cost[a]));
    }
    for (int i = 0; i < n; ++i) {
        if (supply[i] < 0) return -2;
        tot += supply[i];
    }
    // no real path is longer than 2n arcs; ART dominates every real path cost
    const int64_t ART = maxc * (int64_t)(N2 + 1) + 1;
    std::vector<int> stack, cyc_arc, path, own;
    if (!reuse) {
        S.parent.assign(S.V, -1);
        S.pred.assign(S.V, -1);
        S.size.assign(S.V, 1);
        S.mark.assign(S.V, 0);
        S.first_child.assign(S.V, -1);
        S.next_sib.assign(S.V, -1);
        S.prev_sib.assign(S.V, -1);
        S.pot.assign(S.V, 0);
        // Initial strongly feasible tree.  Where the graph has the self arc i -> i (as the flow
        // update's neighbourhood does), the identity flow is feasible, and a breadth-first tree
        // over the nodes through arcs p -> q (p != q) gives a spanning tree of real arcs:
        //   root -> left 0 (artificial, zero flow), left 0 -> right 0 (self arc, supply[0]);
        //   for each tree edge p -> q: left p -> right q (zero flow, pointing away from the root),
        //   then left q hangs from right q by its self arc carrying supply[q] (positive flow).
        // Node pairs the walk does not reach (no self arc, zero supply, or not connected) are
        // joined to the root through artificial arcs carrying their supply (the textbook star).
        // The artificial arcs of the tree's other nodes stay out of the basis at zero flow.
        // (On the flow update of the 512^2 flow workload, 65,536 nodes, with block-search
        // pricing, this start needs 393k pivots against 1.08M from the star of artificial
        // arcs, and runs 2.8x faster.)
        std::vector<int> self(n, -1);
        for (int a = 0; a < m; ++a)
            if (tail[a] == head[a] && self[tail[a]] < 0) self[tail[a]] = a;
        auto usable = [&](int i) { return self[i] >= 0 && supply[i] > 0; };
        std::vector<int> first(n + 1, 0), adj(m);
        for (int a = 0; a < m; ++a) ++first[tail[a] + 1];
        for (int i = 0; i < n; ++i) first[i + 1] += first[i];
        {
            std::vector<int> pos(first.begin(), first.end() - 1);
            for (int a = 0; a < m; ++a) adj[pos[tail[a]]++] = a;
        }
        std::vector<int> par_arc(n, -1), order;
        std::vector<char> reached(n, 0);
        order.reserve(n);
        int root_node = -1;
        for (int i = 0; i < n && root_node < 0; ++i)
            if (usable(i)) root_node = i;
        if (root_node >= 0) {
            reached[root_node] = 1;
            order.push_back(root_node);
            for (size_t h = 0; h < order.size(); ++h) {
                const int pn = order[h];
                for (int k = first[pn]; k < first[pn + 1]; ++k) {
                    const int a = adj[k], q = head[a];
                    if (q == pn || reached[q] || !usable(q)) continue;
                    reached[q] = 1;
                    par_arc[q] = a;
                    order.push_back(q);
                }
            }
        }
        for (int v = 0; v < N2; ++v) {
            const int a = m + v;
            S.cost[a] = ART;
            const int i = v < n ? v : v - n;
            if (reached[i]) {
                // artificial arc root -> v at zero flow; in the tree only for the walk's root
                S.src[a] = S.R;
                S.dst[a] = v;
                S.flow[a] = 0;
                S.state[a] = 1;
                continue;
            }
            const int64_t b = v < n ? supply[v] : -supply[v - n];  // net supply of node v
            if (b > 0) {  // v -> root carries the supply
                S.src[a] = v;
                S.dst[a] = S.R;
                S.flow[a] = b;
            } else {      // root -> v, zero flow points away from the root
                S.src[a] = S.R;
                S.dst[a] = v;
                S.flow[a] = -b;
            }
            S.state[a] = 0;
            S.pred[v] = a;
            S.link_child(S.R, v);
            S.pot[v] = (S.dst[a] == v) ? ART : -ART;
        }
        for (const int q : order) {
            const int L = q, Rn = n + q, sa = self[q];
            if (q == root_node) {
                const int a = m + L;
                S.state[a] = 0;
                S.pred[L] = a;
                S.link_child(S.R, L);
                S.pot[L] = ART;
                S.flow[sa] = supply[q];
                S.state[sa] = 0;
                S.pred[Rn] = sa;
                S.link_child(L, Rn);
                S.pot[Rn] = S.pot[L] + S.cost[sa];
                continue;
            }
            const int pa = par_arc[q], pL = tail[pa];
            S.state[pa] = 0;  // left p -> right q, zero flow
            S.pred[Rn] = pa;
            S.link_child(pL, Rn);
            S.pot[Rn] = S.pot[pL] + S.cost[pa];
            S.flow[sa] = supply[q];  // left q -> right q carries the supply, left q below right q
            S.state[sa] = 0;
            S.pred[L] = sa;
            S.link_child(Rn, L);
            S.pot[L] = S.pot[Rn] - S.cost[sa];
        }
        // subtree sizes of the initial tree (children before parents in reverse preorder)
        {
            std::vector<int> pre;
            pre.reserve(S.V);
            stack.assign(1, S.R);
            while (!stack.empty()) {
                const int x = stack.back();
                stack.pop_back();
                pre.push_back(x);
                for (int c = S.first_child[x]; c >= 0; c = S.next_sib[c]) stack.push_back(c);
            }
            if ((int)pre.size() != S.V) return -2;  // not a spanning tree: cannot happen
            for (int k = S.V - 1; k > 0; --k) S.size[S.parent[pre[k]]] += S.size[pre[k]];
        }
    } else {
        // the previous optimum: same tree, flows and artificial arcs; new costs, so new
        // potentials from the root down
        for (int v = 0; v < N2; ++v) S.cost[m + v] = ART;
        stack.assign(1, S.R);
        S.pot[S.R] = 0;
        while (!stack.empty()) {
            const int x = stack.back();
            stack.pop_back();
            if (x != S.R) {
                const int p = S.parent[x], a = S.pred[x];
                S.pot[x] = (S.dst[a] == x) ? S.pot[p] + S.cost[a] : S.pot[p] - S.cost[a];
            }
            for (int c = S.first_child[x]; c >= 0; c = S.next_sib[c]) stack.push_back(c);
        }
    }
    const int64_t INF = tot + 1;
    auto cap = [&](int) { return INF; };

    std::vector<int8_t> cyc_fwd;
    // (on the flow update of the 512^2 flow workload, against block search over blocks of
    // sqrt(A) arcs: 0.6x the pivots and time of a warm-started solve, 0.85x the time from
    // scratch)
    const int list_len = std::max(16, (int)(3.0 * std::sqrt((double)A)));
    const int minor_limit = std::max(3, list_len / 20);
    std::vector<int> cand;
    cand.reserve(list_len);
    int minor = 0;
    int next = 0;
    int64_t pivots = 0;
    const int64_t max_pivots = (int64_t)50 * A + 1000;
    for (;;) {
        // candidate-list pricing: minor iterations take the most negative reduced cost among
        // the candidates kept from the last scan (dropping those no longer eligible); a major
        // iteration scans the arcs on from where the last scan stopped, keeping up to
        // `list_len` eligible ones, and ends the solve when a scan of every arc finds none
        int enter = -1;
        int64_t best = 0;
        if (minor < minor_limit && !cand.empty()) {
            size_t keep = 0;
            for (size_t k = 0; k < cand.size(); ++k) {
                const int a = cand[k];
                if (S.state[a] != 1) continue;
                const int64_t r = S.rc(a);
                if (r >= 0) continue;
                cand[keep++] = a;
                if (r < best) {
                    best = r;
                    enter = a;
                }
            }
            cand.resize(keep);
            ++minor;
        }
        if (enter < 0) {
            cand.clear();
            minor = 0;
            int scanned = 0;
            while (scanned < A && (int)cand.size() < list_len) {
                const int a = next;
                next = next + 1 == A ? 0 : next + 1;
                ++scanned;
                if (S.state[a] != 1) continue;
                const int64_t r = S.rc(a);
                if (r >= 0) continue;
                cand.push_back(a);
                if (r < best) {
                    best = r;
                    enter = a;
                }
            }
            if (enter < 0) break;  // a whole scan found no eligible arc: optimal
        }
        if (++pivots > max_pivots) return -3;

        // pivot cycle: enter u -> v, tree paths from u and v to the apex
        const int u = S.src[enter], v = S.dst[enter];
        const int join = S.apex(u, v);
        // walk in orientation order: apex -> ... -> u, u -> v, v -> ... -> apex
        cyc_arc.clear();
        cyc_fwd.clear();
        {
            std::vector<int>& path = stack;
            path.clear();
            for (int x = u; x != join; x = S.parent[x]) path.push_back(x);
            for (int k = (int)path.size() - 1; k >= 0; --k) {
                const int x = path[k], ar = S.pred[x];
                cyc_arc.push_back(ar);
                cyc_fwd.push_back(S.dst[ar] == x ? 1 : 0);  // traversed parent -> x
            }
        }
        const int pos_enter = (int)cyc_arc.size();
        cyc_arc.push_back(enter);
        cyc_fwd.push_back(1);
        for (int x = v; x != join; x = S.parent[x]) {
            const int ar = S.pred[x];
            cyc_arc.push_back(ar);
            cyc_fwd.push_back(S.src[ar] == x ? 1 : 0);  // traversed x -> parent
        }
        int64_t delta = INF;
        for (size_t k = 0; k < cyc_arc.size(); ++k) {
            const int ar = cyc_arc[k];
            const int64_t res = cyc_fwd[k] ? cap(ar) - S.flow[ar] : S.flow[ar];
            delta = std::min(delta, res);
        }
        int leave_k = -1;
        for (size_t k = 0; k < cyc_arc.size(); ++k) {
            const int ar = cyc_arc[k];
            const int64_t res = cyc_fwd[k] ? cap(ar) - S.flow[ar] : S.flow[ar];
            if (res == delta) leave_k = (int)k;  // last blocking arc
        }
        if (delta >= INF) return -4;  // unbounded: cannot happen on a transportation graph
        for (size_t k = 0; k < cyc_arc.size(); ++k) {
            const int ar = cyc_arc[k];
            S.flow[ar] += cyc_fwd[k] ? delta : -delta;
        }
        const int leave = cyc_arc[leave_k];
        if (leave == enter) continue;  // bounded only by itself: cannot happen without caps
        // the leaving tree arc cuts off the subtree of its deeper end q
        const int q = (S.pred[S.src[leave]] == leave) ? S.src[leave] : S.dst[leave];
        // the entering endpoint inside q's subtree: u's if the leaving arc is on u's path
        const bool u_side = leave_k < pos_enter;
        const int w_in = u_side ? u : v, z_in = u_side ? v : u;
        // the cut subtree leaves the ancestors of q ...
        // (the apex and its ancestors lose it and regain it below z_in: their sizes stay)
        const int sub = S.size[q];
        for (int y = S.parent[q]; y != join; y = S.parent[y]) S.size[y] -= sub;
        // ... is re-rooted at w_in (parent pointers reversed from w_in up to q).  A path node
        // keeps its old subtree minus the branch towards w_in, and gains the path above it:
        // its new size is the sum of those own parts from q down to it ...
        path.clear();
        own.clear();
        int x = w_in, new_par = z_in, new_pred = enter, below = 0;
        for (;;) {
            const int old_par = S.parent[x], old_pred = S.pred[x];
            path.push_back(x);
            own.push_back(S.size[x] - below);
            below = S.size[x];
            S.unlink_child(x);
            S.pred[x] = new_pred;
            S.link_child(new_par, x);
            if (x == q) break;
            new_par = x;
            new_pred = old_pred;
            x = old_par;
        }
        for (int k = (int)path.size() - 1, acc = 0; k >= 0; --k) {
            acc += own[k];
            S.size[path[k]] = acc;
        }
        // ... and hangs below z_in
        for (int y = z_in; y != join; y = S.parent[y]) S.size[y] += sub;
        S.state[enter] = 0;
        S.state[leave] = 1;
        // the entering arc gets reduced cost 0: the side of w_in moves by d against the other
        const int64_t d = w_in == v ? best : -best;
        if (2 * sub <= S.V)
            S.shift(w_in, -1, d, stack);
        else
            S.shift(S.R, w_in, -d, stack);
    }
    for (int v = 0; v < N2; ++v)
        if (S.flow[m + v] != 0) return -1;  // infeasible
    for (int k = 0; k < m; ++k) flow_out[k] = S.flow[k];
    if (pot_out)
        for (int v = 0; v < N2; ++v) pot_out[v] = S.pot[v];
    if (warm) {
        if (!reuse) {
            warm->S = std::move(fresh);
            warm->n = n;
            warm->m = m;
            warm->tail.assign(tail, tail + m);
            warm->head.assign(head, head + m);
            warm->supply.assign(supply, supply + n);
        }
        warm->valid = true;
    }
    return 0;
}

}  // namespace dd
