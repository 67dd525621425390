// Runs the bank-aware layout optimisation (paper_1409_5826_amd/csrc/lds_layout.h)
// on a problem read from stdin and prints the result, for tests/test_lds_layout.py.
//
// input:  n_species lanes slots n_rows iters seed
//         per row: padded n_terms x0 y0 x1 y1 ...
//         per lane: start n_rows r0 r1 ...
//         per row: class
// output: before after
//         cell_of_species (n_species values)
//         per physical lane: start n_rows r0 r1 ...
#include <cstdio>

#include "lds_layout.h"

int main()
{
    asynet::LayoutProblem p;
    int n_rows = 0;
    long long iters = 0;
    unsigned long long seed = 0;
    if (std::scanf("%d %d %d %d %lld %llu", &p.n_species, &p.lanes, &p.slots, &n_rows, &iters,
                   &seed) != 6)
        return 2;
    p.rows.resize(n_rows);
    p.padded.resize(n_rows);
    for (int r = 0; r < n_rows; ++r) {
        int n = 0;
        if (std::scanf("%d %d", &p.padded[r], &n) != 2)
            return 2;
        for (int e = 0; e < n; ++e) {
            int x = 0, y = 0;
            if (std::scanf("%d %d", &x, &y) != 2)
                return 2;
            p.rows[r].push_back({x, y});
        }
    }
    p.lane_rows.resize(p.lanes);
    p.lane_start.resize(p.lanes);
    for (int l = 0; l < p.lanes; ++l) {
        int n = 0;
        if (std::scanf("%d %d", &p.lane_start[l], &n) != 2)
            return 2;
        p.lane_rows[l].resize(n);
        for (int e = 0; e < n; ++e)
            if (std::scanf("%d", &p.lane_rows[l][e]) != 1)
                return 2;
    }
    p.row_class.resize(n_rows);
    for (int r = 0; r < n_rows; ++r)
        if (std::scanf("%d", &p.row_class[r]) != 1)
            return 2;
    const asynet::LayoutResult res = asynet::optimise_gather_layout(p, iters, seed);
    std::printf("%lld %lld\n", (long long)res.cycles_before, (long long)res.cycles_after);
    for (int c : res.cell_of_species)
        std::printf("%d ", c);
    std::printf("\n");
    for (int l = 0; l < p.lanes; ++l) {
        std::printf("%d %d", res.lane_start[l], (int)res.lane_rows[l].size());
        for (int r : res.lane_rows[l])
            std::printf(" %d", r);
        std::printf("\n");
    }
    return 0;
}
