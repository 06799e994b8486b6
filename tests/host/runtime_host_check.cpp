// Host-only checks of the batch/server building blocks (arena allocator,
// stream assignment and the race check of batch plans). Prints "ok" and exits 0, or names the first failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "hull_host.h"

using hullmi::Arena;

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                          \
        }                                                          \
    } while (0)

static void arena_basic()
{
    Arena a(4096, 256);
    CHECK(a.size() == 4096);
    const size_t x = a.alloc(1);        // rounds up to 256
    const size_t y = a.alloc(1000);     // 1024
    const size_t z = a.alloc(2816);     // the rest exactly
    CHECK(x == 0 && y == 256 && z == 1280);
    CHECK(a.in_use() == 4096 && a.alloc(1) == Arena::kNone && !a.fits(1));
    CHECK(a.release(y));
    CHECK(!a.release(y));               // twice is refused
    CHECK(!a.release(12345));           // never handed out
    CHECK(a.fits(1024) && !a.fits(1025));
    CHECK(a.release(x));                // merges with y's block
    CHECK(a.free_blocks() == 1 && a.fits(1280) && !a.fits(1281));
    CHECK(a.release(z));                // everything merged back
    CHECK(a.free_blocks() == 1 && a.in_use() == 0 && a.peak() == 4096 && a.fits(4096));
    CHECK(a.alloc(4097) == Arena::kNone);
}

// Random alloc/release against a brute-force model of the occupied bytes.
static void arena_random()
{
    const size_t size = 1 << 20, align = 256;
    Arena a(size, align);
    std::vector<char> used(size / align, 0);
    std::vector<std::pair<size_t, size_t>> live;
    std::mt19937_64 rng(12345);
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3) {
            const size_t bytes = 1 + rng() % (size / 16);
            const size_t units = (bytes + align - 1) / align;
            // brute force: does any run of `units` free units exist?
            size_t run = 0;
            bool exists = false;
            for (char u : used) {
                run = u ? 0 : run + 1;
                if (run >= units) { exists = true; break; }
            }
            const size_t off = a.alloc(bytes);
            CHECK((off != Arena::kNone) == exists);
            if (off == Arena::kNone) continue;
            CHECK(off % align == 0 && off + units * align <= size);
            for (size_t k = off / align; k < off / align + units; ++k) {
                CHECK(!used[k]);        // no overlap with a live block
                used[k] = 1;
            }
            live.push_back({off, units});
        } else {
            const size_t i = rng() % live.size();
            CHECK(a.release(live[i].first));
            for (size_t k = live[i].first / align; k < live[i].first / align + live[i].second; ++k)
                used[k] = 0;
            live.erase(live.begin() + i);
        }
        size_t in_use = 0;
        for (char u : used) in_use += u;
        CHECK(a.in_use() == in_use * align);
        CHECK(a.live_blocks() == live.size());
    }
    for (auto &l : live) CHECK(a.release(l.first));
    CHECK(a.in_use() == 0 && a.free_blocks() == 1);
}

static void assign()
{
    // longest first onto the least loaded stream
    std::vector<double> c = {1, 9, 4, 7, 2, 2};
    std::vector<int> s = hullmi::assign_streams(c, 2);
    // order 9(s0) 7(s1) 4(s1: 7<9? no, 11 vs 9) ...
    double load[2] = {0, 0};
    for (size_t j = 0; j < c.size(); ++j) load[s[j]] += c[j];
    CHECK(s[1] == 0 && s[3] == 1);
    CHECK(load[0] + load[1] == 25 && std::abs(load[0] - load[1]) <= 1);
    // one stream takes everything; more streams than jobs leaves some idle
    for (int v : hullmi::assign_streams(c, 1)) CHECK(v == 0);
    std::vector<int> w = hullmi::assign_streams({5, 5, 5}, 8);
    CHECK(w[0] == 0 && w[1] == 1 && w[2] == 2);
    CHECK(hullmi::assign_streams({}, 4).empty());
}

// The race check of batch plans: overlapping byte ranges of different jobs
// where one is written, against a brute-force pairwise test on random spans.
static void spans()
{
    using hullmi::Span;
    CHECK(!hullmi::spans_conflict({}));
    // reads may share memory, writes may not; touching ends do not overlap
    CHECK(!hullmi::spans_conflict({{0, 100, 0, false}, {50, 150, 1, false}}));
    CHECK(hullmi::spans_conflict({{0, 100, 0, false}, {99, 150, 1, true}}));
    CHECK(!hullmi::spans_conflict({{0, 100, 0, true}, {100, 150, 1, true}}));
    CHECK(!hullmi::spans_conflict({{0, 100, 0, true}, {50, 60, 0, true}}));   // one job
    CHECK(!hullmi::spans_conflict({{0, 0, 0, true}, {0, 10, 1, true}}));      // empty
    CHECK(hullmi::spans_conflict({{0, 1000, 0, true}, {10, 20, 1, false}, {5, 6, 2, false}}));
    std::mt19937_64 rng(777);
    for (int it = 0; it < 2000; ++it) {
        std::vector<Span> v;
        const int n = 1 + (int)(rng() % 12);
        for (int i = 0; i < n; ++i) {
            const uintptr_t b = rng() % 1000, len = rng() % 80;
            v.push_back(Span{b, b + len, (int)(rng() % 4), (rng() % 3) == 0});
        }
        bool want = false;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (i != j && v[i].job != v[j].job && (v[i].write || v[j].write) &&
                    v[i].begin < v[i].end && v[j].begin < v[j].end &&
                    v[i].begin < v[j].end && v[j].begin < v[i].end)
                    want = true;
        CHECK(hullmi::spans_conflict(v) == want);
    }
}

int main()
{
    arena_basic();
    arena_random();
    assign();
    spans();
    std::printf("ok\n");
    return 0;
}
