// Runs the host atom decomposition (csrc/partition.cpp) on clouds of many
// sizes and part counts, degenerate lattices and invalid arguments, for a
// build with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitizers.py); checks that every output is a valid partition.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "partition.hpp"

static int failures = 0;
#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

static double urand(unsigned &s)
{
    s = s * 1103515245u + 12345u;
    return ((s >> 8) & 0xFFFFFF) / 16777216.0;
}

static void run(int n, int parts, bool weighted, bool lattice, unsigned seed)
{
    std::vector<double> pos(3 * size_t(n)), w(n);
    for (int i = 0; i < n; ++i) {
        for (int x = 0; x < 3; ++x) pos[3 * i + x] = lattice ? double((i >> (2 * x)) & 3) : 20.0 * urand(seed);
        w[i] = 0.05 + urand(seed);
    }
    // (order and part may not be NULL even for no atoms: at least one entry)
    std::vector<int32_t> order(n > 0 ? n : 1), part(n > 0 ? n : 1), start(parts + 1);
    const char *err = hartree::bisect_atoms(n, n ? pos.data() : nullptr, weighted ? w.data() : nullptr, parts,
                                            order.data(), part.data(), start.data());
    if (err) std::fprintf(stderr, "n %d parts %d: %s\n", n, parts, err);
    CHECK(err == nullptr);
    if (err) return;
    CHECK(start[0] == 0 && start[parts] == n);
    std::vector<int> seen(n, 0);
    for (int p = 0; p < parts; ++p) {
        CHECK(start[p] <= start[p + 1]);
        for (int k = start[p]; k < start[p + 1]; ++k) {
            const int a = order[k];
            CHECK(a >= 0 && a < n);
            if (a < 0 || a >= n) continue;
            seen[a] += 1;
            CHECK(part[a] == p);
        }
    }
    for (int i = 0; i < n; ++i) CHECK(seen[i] == 1);
}

int main()
{
    unsigned seed = 19;
    const int sizes[] = {0, 1, 2, 5, 26, 257, 1000};
    const int parts[] = {1, 2, 3, 7, 19, 64, 1500};
    for (int n : sizes)
        for (int p : parts)
            for (int wt = 0; wt < 2; ++wt) run(n, p, wt != 0, false, seed++);
    run(64, 5, false, true, 1);   // a lattice: degenerate inertia tensors and equal projections
    run(64, 64, true, true, 2);
    // invalid arguments are reported, not crashed on
    std::vector<double> pos = {0, 0, 0, 1, 1, 1};
    std::vector<int32_t> order(2), part(2), start(3);
    CHECK(hartree::bisect_atoms(-1, pos.data(), nullptr, 2, order.data(), nullptr, nullptr) != nullptr);
    CHECK(hartree::bisect_atoms(2, pos.data(), nullptr, 0, order.data(), nullptr, nullptr) != nullptr);
    CHECK(hartree::bisect_atoms(2, nullptr, nullptr, 2, order.data(), nullptr, nullptr) != nullptr);
    std::vector<double> badw = {1.0, -1.0};
    CHECK(hartree::bisect_atoms(2, pos.data(), badw.data(), 2, order.data(), part.data(), start.data()) != nullptr);
    pos[4] = NAN;
    CHECK(hartree::bisect_atoms(2, pos.data(), nullptr, 2, order.data(), part.data(), start.data()) != nullptr);
    if (failures) return 1;
    std::printf("partition sanitizer driver: ok\n");
    return 0;
}
