// Host test of the serving arena: random alloc/release sequences checked against a
// brute-force byte map (no two live ranges overlap, every range is inside the block, the
// free list is coalesced, and a full release returns one free range of full size).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2011_03479_amd/csrc/arena.h"

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main() {
    using gempe::Arena;
    {
        Arena a(1000, 256);  // capacity rounds down to 768
        CHECK(a.capacity() == 768);
        size_t x = a.alloc(1);
        CHECK(x == 0);
        size_t y = a.alloc(300);  // 512 bytes
        CHECK(y == 256);
        CHECK(a.alloc(1) == Arena::kNone);
        CHECK(a.used() == 768 && a.peak() == 768);
        CHECK(a.release(x));
        CHECK(!a.release(x));
        CHECK(a.alloc(257) == Arena::kNone);  // only 256 free
        CHECK(a.release(y));
        CHECK(a.free_ranges() == 1 && a.largest_free() == 768 && a.used() == 0);
        CHECK(a.alloc(768) == 0);
    }
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 20; ++trial) {
        const size_t cap = 256 * (64 + rng() % 512);
        Arena a(cap, 256);
        std::vector<int> owner(cap / 256, -1);
        std::vector<std::pair<size_t, size_t>> live;  // offset, rounded size
        for (int step = 0; step < 5000; ++step) {
            if (live.empty() || rng() % 3 != 0) {
                size_t want = 1 + rng() % (cap / 8);
                size_t off = a.alloc(want);
                size_t need = a.round(want);
                if (off == Arena::kNone) {
                    // first fit must really have failed: no free run of `need` bytes
                    size_t run = 0, best = 0;
                    for (size_t k = 0; k < owner.size(); ++k) {
                        run = owner[k] < 0 ? run + 256 : 0;
                        if (run > best) best = run;
                    }
                    CHECK(best < need);
                    CHECK(a.largest_free() == best);
                    continue;
                }
                CHECK(off % 256 == 0 && off + need <= cap);
                for (size_t k = off / 256; k < (off + need) / 256; ++k) {
                    CHECK(owner[k] < 0);
                    owner[k] = step;
                }
                live.push_back({off, need});
            } else {
                size_t idx = rng() % live.size();
                auto [off, need] = live[idx];
                CHECK(a.release(off));
                for (size_t k = off / 256; k < (off + need) / 256; ++k) owner[k] = -1;
                live[idx] = live.back();
                live.pop_back();
            }
            size_t used = 0;
            for (auto &l : live) used += l.second;
            CHECK(a.used() == used && a.live_count() == live.size());
        }
        for (auto &l : live) CHECK(a.release(l.first));
        CHECK(a.used() == 0 && a.free_ranges() == 1 && a.largest_free() == a.capacity());
    }
    std::printf("arena ok\n");
    return 0;
}
