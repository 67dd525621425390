// Bank-aware placement for the packed-rows gathers (host code).
//
// Every slot of the packed layout is two gather instructions (the x and the
// y factor of each lane's term), and the cells a wave gathers are the same for
// every zone and every step.  gfx950 serves an 8-byte LDS read in two halves
// of 32 lanes; a half takes as many cycles as the most distinct addresses
// that fall on one of the 64 four-byte banks (equal addresses are broadcast),
// so with 8-byte cells two different cells collide when their indices agree
// modulo 32.  A 4-byte read is served the same way over 32 banks, so 4-byte
// cells collide under the same rule and one placement serves both precisions.  The packing leaves three things free that change nothing in the
// arithmetic: which Y cell holds which species, which physical lane holds
// which lane's column, and the order of the rows within a lane (each row is
// still summed in its own order into its own cell).  A seeded simulated
// annealing over these three minimises the summed cycles of all gather
// half-instructions.  Two constraints keep the packing's one-factor blocks
// intact: columns move only between the halves of one wave, and rows swap
// only with rows of the same class.  The result is deterministic for a given
// input.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace asynet {

struct LayoutProblem {
    int n_species = 0;  // cells 0..N-1 hold species (permuted), cell N the constant 1.0
    int lanes = 0;      // 64 * waves
    int slots = 0;      // C, a multiple of 4
    // per packed row: the (x, y) factors of its terms, species indices (N = the 1.0 cell)
    std::vector<std::vector<std::pair<int, int>>> rows;
    std::vector<int> padded;               // per row: its slot count
    std::vector<std::vector<int>> lane_rows;  // per lane: its rows in slot order
    std::vector<int> lane_start;              // per lane: slot of its first row (padding before)
    std::vector<int> row_class;               // per row: rows swap only within a class
};

struct LayoutResult {
    std::vector<int> cell_of_species;         // [N]: Y cell of each species
    std::vector<std::vector<int>> lane_rows;  // per physical lane: rows in slot order
    std::vector<int> lane_start;              // per physical lane: slot of its first row
    int64_t cycles_before = 0, cycles_after = 0;  // modelled gather half-instruction cycles
};

class GatherAnneal {
  public:
    static constexpr int kHalf = 32;   // lanes served together
    static constexpr int kBanks = 32;  // 8-byte cells: bank pair = cell mod 32

    explicit GatherAnneal(const LayoutProblem &p) : p_(p)
    {
        N_ = p.n_species;
        L_ = p.lanes;
        C_ = p.slots;
        H_ = L_ / kHalf;
        K_ = 2 * C_ * H_;
        lr_ = p.lane_rows;
        col_.assign(L_, std::vector<int>(2 * C_, N_));
        for (int k = 0; k < L_; ++k)
            fill_col(k);
        pos_.resize(L_);
        for (int k = 0; k < L_; ++k)
            pos_[k] = k;
        place_.resize(N_ + 1);
        for (int i = 0; i <= N_; ++i)
            place_[i] = i;
        mult_.assign((size_t)K_ * (N_ + 1), 0);
        bank_.assign((size_t)K_ * kBanks, 0);
        cost_.assign(K_, 0);
        for (int k = 0; k < L_; ++k)
            for (int a = 0; a < 2; ++a)
                for (int s = 0; s < C_; ++s)
                    add(inst(a, s, pos_[k] / kHalf), col_[k][a * C_ + s]);
        total_ = 0;
        for (int q = 0; q < K_; ++q)
            total_ += (cost_[q] = max_bank(q));
    }

    int64_t total() const { return total_; }

    void run(int64_t iters, uint64_t seed)
    {
        rng_ = seed ? seed : 0x9e3779b97f4a7c15ull;
        const double T0 = 1.5, T1 = 0.02;
        std::vector<int> touched;
        for (int64_t it = 0; it < iters; ++it) {
            const double T = T0 + (T1 - T0) * (double)it / (double)iters;
            const uint32_t mv = next() % 10;
            if (mv < 4)
                try_place(T, touched);
            else if (mv < 7)
                try_lane(T, touched);
            else
                try_order(T, touched);
        }
    }

    LayoutResult result(int64_t before) const
    {
        LayoutResult r;
        r.cell_of_species.assign(place_.begin(), place_.begin() + N_);
        r.lane_rows.assign(L_, {});
        r.lane_start.assign(L_, 0);
        for (int k = 0; k < L_; ++k) {
            r.lane_rows[pos_[k]] = lr_[k];
            r.lane_start[pos_[k]] = p_.lane_start[k];
        }
        r.cycles_before = before;
        r.cycles_after = total_;
        return r;
    }

  private:
    const LayoutProblem &p_;
    int N_, L_, C_, H_, K_;
    std::vector<std::vector<int>> lr_;   // per lane column k: its rows
    std::vector<std::vector<int>> col_;  // per lane column: x cells [0, C), y cells [C, 2C)
    std::vector<int> pos_;               // physical lane of column k
    std::vector<int> place_;             // cell of species (place_[N] = N)
    std::vector<uint16_t> mult_;         // [inst][species]: lanes gathering it
    std::vector<uint16_t> bank_;         // [inst][bank]: distinct species on it
    std::vector<int> cost_;              // [inst]: cycles
    int64_t total_ = 0;
    uint64_t rng_ = 0;

    uint64_t next()
    {
        rng_ ^= rng_ >> 12;
        rng_ ^= rng_ << 25;
        rng_ ^= rng_ >> 27;
        return rng_ * 0x2545f4914f6cdd1dull;
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    bool accept(int delta, double T) { return delta <= 0 || uniform() < std::exp(-delta / T); }

    int inst(int a, int s, int h) const { return (a * C_ + s) * H_ + h; }
    int bank_of(int species) const { return place_[species] % kBanks; }

    void fill_col(int k)
    {
        std::vector<int> &c = col_[k];
        std::fill(c.begin(), c.end(), N_);
        int s = p_.lane_start[k];
        for (int r : lr_[k]) {
            const auto &t = p_.rows[r];
            for (size_t e = 0; e < t.size(); ++e) {
                c[s + e] = t[e].first;
                c[C_ + s + e] = t[e].second;
            }
            s += p_.padded[r];
        }
    }
    void add(int q, int sp)
    {
        if (mult_[(size_t)q * (N_ + 1) + sp]++ == 0)
            ++bank_[(size_t)q * kBanks + bank_of(sp)];
    }
    void remove(int q, int sp)
    {
        if (--mult_[(size_t)q * (N_ + 1) + sp] == 0)
            --bank_[(size_t)q * kBanks + bank_of(sp)];
    }
    int max_bank(int q) const
    {
        const uint16_t *b = &bank_[(size_t)q * kBanks];
        return *std::max_element(b, b + kBanks);
    }
    // re-cost the touched instructions; returns the change of the total
    int recost(std::vector<int> &touched, std::vector<int> &old)
    {
        std::sort(touched.begin(), touched.end());
        touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
        old.resize(touched.size());
        int delta = 0;
        for (size_t t = 0; t < touched.size(); ++t) {
            old[t] = cost_[touched[t]];
            const int c = max_bank(touched[t]);
            delta += c - old[t];
            cost_[touched[t]] = c;
        }
        return delta;
    }
    void restore_costs(const std::vector<int> &touched, const std::vector<int> &old)
    {
        for (size_t t = 0; t < touched.size(); ++t)
            cost_[touched[t]] = old[t];
    }

    void swap_place(int i, int j)
    {
        // move the bank counts of every instruction that gathers i or j
        const int bi = bank_of(i), bj = bank_of(j);
        for (int q = 0; q < K_; ++q) {
            const bool hi = mult_[(size_t)q * (N_ + 1) + i] > 0;
            const bool hj = mult_[(size_t)q * (N_ + 1) + j] > 0;
            if (hi == hj)
                continue;  // both or neither: the bank counts do not change
            uint16_t *b = &bank_[(size_t)q * kBanks];
            if (hi) {
                --b[bi];
                ++b[bj];
            } else {
                --b[bj];
                ++b[bi];
            }
        }
        std::swap(place_[i], place_[j]);
    }
    void try_place(double T, std::vector<int> &touched)
    {
        if (N_ < 2)
            return;
        const int i = (int)(next() % N_), j = (int)(next() % N_);
        if (bank_of(i) == bank_of(j))
            return;
        touched.clear();
        for (int q = 0; q < K_; ++q)
            if ((mult_[(size_t)q * (N_ + 1) + i] > 0) != (mult_[(size_t)q * (N_ + 1) + j] > 0))
                touched.push_back(q);
        swap_place(i, j);
        std::vector<int> old;
        const int delta = recost(touched, old);
        if (accept(delta, T)) {
            total_ += delta;
        } else {
            swap_place(i, j);
            restore_costs(touched, old);
        }
    }

    void move_lane(int k, int from_h, int to_h)
    {
        for (int a = 0; a < 2; ++a)
            for (int s = 0; s < C_; ++s) {
                const int sp = col_[k][a * C_ + s];
                remove(inst(a, s, from_h), sp);
                add(inst(a, s, to_h), sp);
            }
    }
    void try_lane(double T, std::vector<int> &touched)
    {
        if (H_ < 2)
            return;
        const int k1 = (int)(next() % L_), k2 = (int)(next() % L_);
        const int h1 = pos_[k1] / kHalf, h2 = pos_[k2] / kHalf;
        if (h1 == h2 || pos_[k1] / 64 != pos_[k2] / 64)
            return;
        move_lane(k1, h1, h2);
        move_lane(k2, h2, h1);
        touched.clear();
        for (int a = 0; a < 2; ++a)
            for (int s = 0; s < C_; ++s) {
                touched.push_back(inst(a, s, h1));
                touched.push_back(inst(a, s, h2));
            }
        std::vector<int> old;
        const int delta = recost(touched, old);
        if (accept(delta, T)) {
            total_ += delta;
            std::swap(pos_[k1], pos_[k2]);
        } else {
            move_lane(k1, h2, h1);
            move_lane(k2, h1, h2);
            restore_costs(touched, old);
        }
    }

    void retarget(int k, const std::vector<int> &from, const std::vector<int> &to,
                  std::vector<int> *touched)
    {
        const int h = pos_[k] / kHalf;
        for (int a = 0; a < 2; ++a)
            for (int s = 0; s < C_; ++s) {
                const int u = from[a * C_ + s], v = to[a * C_ + s];
                if (u == v)
                    continue;
                remove(inst(a, s, h), u);
                add(inst(a, s, h), v);
                if (touched)
                    touched->push_back(inst(a, s, h));
            }
    }
    void try_order(double T, std::vector<int> &touched)
    {
        const int k = (int)(next() % L_);
        const int n = (int)lr_[k].size();
        if (n < 2)
            return;
        const int u = (int)(next() % n), v = (int)(next() % n);
        if (u == v || p_.row_class[lr_[k][u]] != p_.row_class[lr_[k][v]])
            return;
        const std::vector<int> before = col_[k];
        std::swap(lr_[k][u], lr_[k][v]);
        fill_col(k);
        touched.clear();
        retarget(k, before, col_[k], &touched);
        std::vector<int> old;
        const int delta = recost(touched, old);
        if (accept(delta, T)) {
            total_ += delta;
        } else {
            const std::vector<int> after = col_[k];
            std::swap(lr_[k][u], lr_[k][v]);
            col_[k] = before;
            retarget(k, after, before, nullptr);
            restore_costs(touched, old);
        }
    }
};

// Optimise the layout; iterations scale with the number of gather instructions.
inline LayoutResult optimise_gather_layout(const LayoutProblem &p, int64_t iters, uint64_t seed)
{
    GatherAnneal g(p);
    const int64_t before = g.total();
    g.run(iters, seed);
    return g.result(before);
}

}  // namespace asynet
