// Host-only planner exercise, built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_planner_sanitizers.py: every length 1..3000 in every kind (c2c, r2c, c2r,
// DCT-II, DCT-III) and dtype,
// assorted multi-dimensional shapes, and the schedule of a 3000-length ragged batch.
#include "planner.h"
#include <cstdio>
#include <random>
using namespace mifft;
int main()
{
    int fails = 0, plans = 0;
    for (int64_t n = 1; n <= 3000; ++n)
        for (int dt = 0; dt < 4; ++dt)
            for (int kind = 0; kind < 5; ++kind) {
                if (dt >= 2 && kind) continue;
                PlanSpec sp;
                std::string err;
                // c2r inverse; r2c and the DCT kinds forward; c2c alternates
                const int dir = kind == 2 ? 1 : (kind != 0 ? -1 : (n % 2 ? 1 : -1));
                const int st = build_plan(1, &n, 3, kind, dir, dt, sp, err);
                ++plans;
                if (st != 0) { ++fails; std::printf("fail n=%lld dt=%d kind=%d: %s\n", (long long)n, dt, kind, err.c_str()); }
                else (void)sp.describe();
            }
    const int64_t md[][3] = {{4, 6, 1}, {17, 20, 1}, {512, 512, 512}, {97, 101, 3}, {1, 1, 1}, {4096, 4096, 1}, {30, 1024, 7}};
    for (auto &d : md)
        for (int rank = 1; rank <= 3; ++rank)
            for (int kind = 0; kind < 3; ++kind) {
                PlanSpec sp;
                std::string err;
                const int st = build_plan(rank, d, 2, kind, kind == 2 ? 1 : -1, 0, sp, err);
                ++plans;
                if (st != 0) std::printf("md fail %lld %lld %lld rank %d kind %d: %s\n", (long long)d[0], (long long)d[1], (long long)d[2], rank, kind, err.c_str());
            }
    std::mt19937_64 rng(5);
    std::vector<int64_t> L(3000);
    for (auto &x : L) x = 64 + int64_t(rng() % 65472);
    ManySpec ms;
    RaggedSchedule rs;
    std::string err;
    int st = build_many(int64_t(L.size()), L.data(), 0, -1, 0, ms, err);
    if (st == 0) st = schedule_many(ms, rs, err);
    std::printf("plans=%d fails=%d ragged st=%d blocks=%zu %s\n", plans, fails, st, rs.blocks.size(), err.c_str());
    return fails != 0 || st != 0;
}
