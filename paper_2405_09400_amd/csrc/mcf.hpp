// Host integer min-cost flow (network simplex) used by the flow update.
#pragma once

#include <cstdint>

namespace dd {

// Bipartite transportation problem: left node i supplies supply[i], right node j demands
// supply[j]; arcs tail[a] -> head[a] with integer cost, no upper bound.  Writes optimal flows
// and (if pot_out) node potentials (left 0..n-1, right n..2n-1) with reduced cost
// cost[a] + pot[tail] - pot[n + head] >= 0, and == 0 where flow > 0.
// Returns 0, -1 infeasible, -2 bad input, -3 pivot limit, -4 unbounded.
int mcf_network_simplex(int n, int m, const int32_t* tail, const int32_t* head,
                        const int64_t* cost, const int64_t* supply, int64_t* flow_out,
                        int64_t* pot_out);

// The same with a kept state: when the graph and the supplies equal those of the last
// successful solve kept in `warm`, that solve's optimal basis (tree and flows) is the start
// and only the potentials are rebuilt for the new costs; the solve is then kept in `warm`.
// warm may be null.
struct McfWarm;
McfWarm* mcf_warm_create();
void mcf_warm_free(McfWarm* w);
int mcf_network_simplex_warm(int n, int m, const int32_t* tail, const int32_t* head,
                             const int64_t* cost, const int64_t* supply, int64_t* flow_out,
                             int64_t* pot_out, McfWarm* warm);

}  // namespace dd
