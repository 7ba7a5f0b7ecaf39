// Host-only checks of the evaluation server's staging arena and admission
// policy (server_admission.hpp).  Prints one line per failed check and
// "checks passed" at the end; exit status 1 on any failure.
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "server_admission.hpp"

using nebem::Arena;
using nebem::AdmitState;

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);                  \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

struct Req {
    int64_t id = 0;
    size_t bytes = 0, off = 0;
    bool large = false;
    bool live = false;
};

// every live request lies inside the arena, 256-aligned, and no two overlap
static bool disjoint(const std::vector<Req> &rs, size_t size)
{
    for (size_t i = 0; i < rs.size(); ++i) {
        if (!rs[i].live) continue;
        const size_t a0 = rs[i].off, a1 = a0 + nebem::arena_bytes(rs[i].bytes);
        if (a0 % 256 || a1 > size) return false;
        for (size_t j = i + 1; j < rs.size(); ++j) {
            if (!rs[j].live) continue;
            const size_t b0 = rs[j].off, b1 = b0 + nebem::arena_bytes(rs[j].bytes);
            if (a0 < b1 && b0 < a1) return false;
        }
    }
    return true;
}

static void arena_basics()
{
    Arena a;
    a.init(10000);  // rounded down to 39 granules
    CHECK(a.size == 9984);
    size_t o1, o2, o3;
    CHECK(a.alloc(1, o1) && o1 == 0);
    CHECK(a.alloc_top(300, o2) && o2 == 9984 - 512);
    CHECK(a.alloc(256, o3) && o3 == 256);
    size_t big;
    CHECK(!a.alloc(9984, big));
    a.release(o1, 1);
    a.release(o3, 256);
    a.release(o2, 300);
    CHECK(a.free_.size() == 1 && a.free_.begin()->first == 0 && a.free_.begin()->second == 9984);
    CHECK(a.alloc(9984, big) && big == 0);
}

static void fcfs_and_backfill()
{
    // arena of 64 granules: small = at most 256 bytes (one granule)
    Arena a;
    a.init(64 * 256);
    AdmitState st;
    std::vector<Req> rs(6);
    for (int k = 0; k < 6; ++k) rs[k].id = k + 1;
    rs[0].bytes = 40 * 256;  // fits
    rs[1].bytes = 30 * 256;  // does not fit beside it: blocked head
    rs[2].bytes = 100;       // small: passes the head
    rs[3].bytes = 2 * 256;   // fits, but not small: waits behind the head
    rs[4].bytes = 256;       // small: passes
    rs[5].bytes = 1;         // small: passes
    std::deque<Req *> q;
    for (auto &r : rs) q.push_back(&r);
    std::vector<int64_t> order;
    auto on = [&](Req *r) {
        r->live = true;
        order.push_back(r->id);
    };
    CHECK(nebem::admit(q, a, st, 0, on));
    CHECK((order == std::vector<int64_t>{1, 3, 5, 6}));
    CHECK(q.size() == 2 && q[0]->id == 2 && q[1]->id == 4);
    CHECK(st.blocked_id == 2 && st.bypassed == 3 && st.backfilled == 3);
    CHECK(rs[0].off == 0);
    CHECK(rs[2].off >= 61 * 256 && rs[4].off >= 61 * 256 && rs[5].off >= 61 * 256);  // at the top
    CHECK(disjoint(rs, a.size));
    // the large one finishes: the head and then the one behind it enter
    a.release(rs[0].off, rs[0].bytes);
    rs[0].live = false;
    order.clear();
    CHECK(nebem::admit(q, a, st, 0, on));
    CHECK((order == std::vector<int64_t>{2, 4}));
    CHECK(q.empty() && st.blocked_id == 0);
    CHECK(disjoint(rs, a.size));
}

static void bypass_cap()
{
    Arena a;
    a.init(64 * 256);
    AdmitState st;
    std::vector<Req> rs(2 + nebem::kMaxBypass + 5);
    for (size_t k = 0; k < rs.size(); ++k) {
        rs[k].id = (int64_t)k + 1;
        rs[k].bytes = 16;
    }
    rs[0].bytes = 63 * 256;  // fills all but one granule
    rs[1].bytes = 2 * 256;   // blocked head
    std::deque<Req *> q;
    for (auto &r : rs) q.push_back(&r);
    int admitted = 0;
    auto on = [&](Req *r) {
        r->live = true;
        ++admitted;
    };
    nebem::admit(q, a, st, 0, on);
    CHECK(admitted == 2);  // the big one and one small one in the last granule
    // the small ones keep finishing; the head stays blocked while the big
    // one runs, and after kMaxBypass of them no more pass it
    for (int round = 0; round < 2 * nebem::kMaxBypass; ++round) {
        for (auto &r : rs)
            if (r.live && r.id > 2) {
                a.release(r.off, r.bytes);
                r.live = false;
            }
        nebem::admit(q, a, st, 0, on);
        CHECK(disjoint(rs, a.size));
    }
    CHECK(st.bypassed == nebem::kMaxBypass && st.blocked_id == 2);
    CHECK(admitted == 1 + nebem::kMaxBypass);
    CHECK(q.size() == rs.size() - 1 - nebem::kMaxBypass && q.front()->id == 2);
    // the big one finishes: the head enters first, then the rest
    for (auto &r : rs)
        if (r.live) {
            a.release(r.off, r.bytes);
            r.live = false;
        }
    std::vector<int64_t> order;
    nebem::admit(q, a, st, 0, [&](Req *r) {
        r->live = true;
        order.push_back(r->id);
    });
    CHECK(!order.empty() && order[0] == 2);
    CHECK(q.empty() && st.blocked_id == 0);
}

static void large_cap()
{
    // room for everything; at most one large request at a time
    Arena a;
    a.init(64 * 256);
    AdmitState st;
    std::vector<Req> rs(5);
    for (int k = 0; k < 5; ++k) {
        rs[k].id = k + 1;
        rs[k].bytes = 256;
    }
    rs[0].large = rs[1].large = rs[3].large = true;
    std::deque<Req *> q;
    for (auto &r : rs) q.push_back(&r);
    std::vector<int64_t> order;
    auto on = [&](Req *r) {
        r->live = true;
        order.push_back(r->id);
    };
    nebem::admit(q, a, st, 1, on);
    CHECK((order == std::vector<int64_t>{1, 3, 5}));  // 2 waits at the head, 3 and 5 pass, 4 is large
    CHECK(st.active_large == 1 && st.blocked_id == 2 && st.backfilled == 2);
    // the large one finishes (the caller's part: release and decrement)
    a.release(rs[0].off, rs[0].bytes);
    rs[0].live = false;
    --st.active_large;
    order.clear();
    nebem::admit(q, a, st, 1, on);
    CHECK((order == std::vector<int64_t>{2}));
    CHECK(st.active_large == 1 && q.size() == 1 && q[0]->id == 4);
    // without a cap all of them enter at once
    Arena b;
    b.init(64 * 256);
    AdmitState st2;
    std::vector<Req> rs2 = rs;
    std::deque<Req *> q2;
    for (auto &r : rs2) {
        r.live = false;
        q2.push_back(&r);
    }
    int n = 0;
    nebem::admit(q2, b, st2, 0, [&](Req *) { ++n; });
    CHECK(n == 5 && st2.active_large == 3 && st2.backfilled == 0);
}

static void random_traffic(int max_large)
{
    std::mt19937_64 g(7);
    Arena a;
    a.init(1 << 20);
    AdmitState st;
    std::vector<Req> rs(4000);
    std::deque<Req *> q;
    size_t next = 0;
    int64_t admitted = 0;
    auto on = [&](Req *r) {
        r->live = true;
        ++admitted;
    };
    auto release_all = [&] {
        for (auto &r : rs)
            if (r.live) {
                a.release(r.off, r.bytes);
                r.live = false;
                if (r.large) --st.active_large;
            }
    };
    for (int step = 0; step < 20000; ++step) {
        if (next < rs.size() && g() % 4 == 0) {
            Req &r = rs[next];
            r.id = (int64_t)next + 1;
            // log-uniform sizes from 1 byte to half the arena
            const double u = std::uniform_real_distribution<double>(0.0, 1.0)(g);
            r.bytes = (size_t)std::exp(u * std::log((double)(1 << 20) / 2.0)) + 1;
            r.large = r.bytes > (1u << 14);
            q.push_back(&r);
            ++next;
        }
        for (size_t k = 0; k < next; ++k)
            if (rs[k].live && g() % 16 == 0) {
                a.release(rs[k].off, rs[k].bytes);
                rs[k].live = false;
                if (rs[k].large) --st.active_large;
            }
        nebem::admit(q, a, st, max_large, on);
        if (step % 97 == 0) CHECK(disjoint(rs, a.size));
        CHECK(st.bypassed <= nebem::kMaxBypass);
        CHECK(max_large <= 0 || st.active_large <= max_large);
    }
    CHECK(disjoint(rs, a.size));
    // drain: whatever is queued enters once the arena empties
    for (int k = 0; k < 4000 && !q.empty(); ++k) {
        release_all();
        nebem::admit(q, a, st, max_large, on);
    }
    CHECK(q.empty() && admitted == (int64_t)next && next == rs.size());
    CHECK(st.backfilled > 0);
    release_all();
    CHECK(a.free_.size() == 1 && a.free_.begin()->second == a.size && st.active_large == 0);
}

int main()
{
    arena_basics();
    fcfs_and_backfill();
    bypass_cap();
    large_cap();
    random_traffic(0);
    random_traffic(2);
    if (failures) return 1;
    std::printf("checks passed\n");
    return 0;
}
