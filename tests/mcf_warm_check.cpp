// Host check of the warm-started min-cost flow: a sequence of problems on one graph with one
// set of supplies and changing costs, each solved from the previous optimum, must reach the
// optimal value of a solve from scratch and satisfy the optimality conditions.
#include <cstdio>
#include <cstdint>
#include <random>
#include <vector>

#include "mcf.hpp"

int main() {
    std::mt19937_64 rng(7);
    int bad = 0;
    for (int inst = 0; inst < 6; ++inst) {
        const int M = 6 + inst * 3, n = M * M;
        std::vector<int32_t> tail, head;
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                const int p = i * M + j;
                const int d[5][2] = {{-1, 0}, {0, -1}, {0, 0}, {0, 1}, {1, 0}};
                for (const auto& e : d) {
                    const int a = i + e[0], b = j + e[1];
                    if (a < 0 || a >= M || b < 0 || b >= M) continue;
                    tail.push_back(p);
                    head.push_back(a * M + b);
                }
            }
        const int m = (int)tail.size();
        std::vector<int64_t> supply(n);
        std::uniform_int_distribution<int64_t> us(inst % 2 ? 0 : 1, 1 << 20);
        for (auto& v : supply) v = us(rng);
        dd::McfWarm* warm = dd::mcf_warm_create();
        std::normal_distribution<double> nd;
        std::vector<double> base(m);
        for (auto& v : base) v = nd(rng);
        for (int round = 0; round < 5; ++round) {
            std::vector<int64_t> cost(m);
            for (int a = 0; a < m; ++a)
                cost[a] = tail[a] == head[a] ? 0 : (int64_t)((base[a] + 0.3 * nd(rng)) * (1 << 20));
            std::vector<int64_t> fw(m), fc(m), pw(2 * n);
            const int rw = dd::mcf_network_simplex_warm(n, m, tail.data(), head.data(), cost.data(),
                                                        supply.data(), fw.data(), pw.data(), warm);
            const int rc = dd::mcf_network_simplex(n, m, tail.data(), head.data(), cost.data(),
                                                   supply.data(), fc.data(), nullptr);
            __int128 vw = 0, vc = 0;
            for (int a = 0; a < m; ++a) {
                vw += (__int128)fw[a] * cost[a];
                vc += (__int128)fc[a] * cost[a];
            }
            // feasibility and complementary slackness of the warm solve
            std::vector<int64_t> out(n, 0), in(n, 0);
            bool ok = rw == 0 && rc == 0 && vw == vc;
            for (int a = 0; a < m; ++a) {
                if (fw[a] < 0) ok = false;
                out[tail[a]] += fw[a];
                in[head[a]] += fw[a];
                const int64_t r = cost[a] + pw[tail[a]] - pw[n + head[a]];
                if (r < 0 || (fw[a] > 0 && r != 0)) ok = false;
            }
            for (int i = 0; i < n; ++i)
                if (out[i] != supply[i] || in[i] != supply[i]) ok = false;
            if (!ok) {
                std::printf("instance %d round %d: warm %d cold %d values %s\n", inst, round, rw, rc,
                            vw == vc ? "equal" : "differ");
                ++bad;
            }
        }
        dd::mcf_warm_free(warm);
    }
    std::printf(bad ? "FAIL\n" : "OK\n");
    return bad ? 1 : 0;
}
