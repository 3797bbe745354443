// Applies every generated merge network (list of KM, batch of 16) to random
// inputs with the kernel's semantics and compares the result with a sort.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <utility>
#include <vector>

#include "kbmi_merge_network.h"

using kbmi::MergeNetwork;

template <int KM>
bool check(std::mt19937_64 &rng, int trials) {
    using Net = MergeNetwork<KM>;
    for (int t = 0; t < trials; ++t) {
        std::vector<uint64_t> r(KM + 16);
        std::vector<float> a(KM + 16);
        for (auto &x : r) x = (rng() >> 2) | 1u;           // distinct non-zero keys (whp)
        std::sort(r.begin(), r.begin() + KM, std::greater<uint64_t>());
        const int empty_list = t % 4 == 0 ? (int)(rng() % (KM + 1)) : 0;
        for (int i = KM - empty_list; i < KM; ++i) r[i] = 0;
        const int empty_batch = (int)(rng() % 17);
        for (int i = 0; i < empty_batch; ++i) r[KM + (rng() % 16)] = 0;
        for (int i = 0; i < KM + 16; ++i) a[i] = (float)(r[i] % 1000003);   // alpha follows its key
        std::vector<uint64_t> want(r);
        std::sort(want.begin(), want.end(), std::greater<uint64_t>());
        for (int k = 0; k < Net::n_ops; ++k) {
            const auto op = Net::ops[k];
            const bool c = r[op.b] > r[op.a];
            if (op.kind == 0) {
                if (c) {
                    std::swap(r[op.a], r[op.b]);
                    std::swap(a[op.a], a[op.b]);
                }
            } else if (c) {
                r[op.a] = r[op.b];
                a[op.a] = a[op.b];
            }
        }
        for (int s = 0; s < KM; ++s) {
            const int p = Net::perm[s];
            if (r[p] != want[s] || a[p] != (float)(want[s] % 1000003)) {
                std::printf("KM=%d trial %d slot %d wrong\n", KM, t, s);
                return false;
            }
        }
    }
    return true;
}

template <int... K>
bool check_all(std::mt19937_64 &rng, std::integer_sequence<int, K...>) {
    return (check<16 + 2 * K>(rng, 2000) && ...);
}

int main() {
    std::mt19937_64 rng(1901);
    const bool ok = check_all(rng, std::make_integer_sequence<int, 25>());
    std::puts(ok ? "merge networks ok" : "merge networks FAILED");
    return ok ? 0 : 1;
}
