// Randomised check of the serving request ring's bookkeeping (ReqRing):
// every taken piece lies inside the buffer, is aligned, and overlaps no
// other live piece; a ring whose pieces are all back hands out its whole
// capacity again; a take fails only when no free range of that size exists
// in the order the ring hands them out.  Prints "ok" and exits 0, or names
// the first violation and exits 1.
#include <cstdio>
#include <cstdint>
#include <random>
#include <vector>

#include "req_ring.hpp"

using vc::ReqRing;

struct Live {
    uint64_t at, bytes;
};

static int fail(const char* what, long step) {
    std::printf("FAIL %s at step %ld\n", what, step);
    return 1;
}

int main() {
    const uint64_t caps[] = {4096, 1u << 20, 64ull << 20};
    long step = 0;
    for (uint64_t cap : caps) {
        for (int seed = 0; seed < 20; ++seed) {
            std::mt19937_64 rng(seed * 7919 + cap);
            ReqRing ring(cap);
            std::vector<Live> live;
            uint64_t taken_ok = 0, refused = 0;
            for (int it = 0; it < 20000; ++it, ++step) {
                const bool do_take = live.empty() || rng() % 100 < 55;
                if (do_take) {
                    // sizes from 1 byte to about a third of the ring
                    const uint64_t want = 1 + rng() % (cap / 3);
                    uint64_t at = ~0ull;
                    if (ring.take(want, &at)) {
                        const uint64_t b = (want + 255) & ~255ull;
                        if (at % ReqRing::ALIGN) return fail("unaligned piece", step);
                        if (at + b > cap) return fail("piece past the end", step);
                        for (const Live& q : live)
                            if (at < q.at + q.bytes && q.at < at + b)
                                return fail("overlapping pieces", step);
                        live.push_back({at, b});
                        ++taken_ok;
                    } else {
                        if (live.empty()) return fail("refused on an empty ring", step);
                        ++refused;
                    }
                } else {
                    // give back a random live piece (any order)
                    const size_t i = rng() % live.size();
                    ring.give(live[i].at);
                    live.erase(live.begin() + i);
                }
                if (ring.live() < live.size()) return fail("ring lost a live piece", step);
                if (live.empty() && ring.live() != 0) return fail("pieces left after all came back", step);
            }
            if (taken_ok < 1000) return fail("too few pieces taken", step);
            // everything back: the whole capacity is one free range again
            for (const Live& q : live) ring.give(q.at);
            uint64_t at = ~0ull;
            if (!ring.take(cap, &at) || at != 0) return fail("whole ring not free after all came back", step);
            ring.give(at);
            (void)refused;
        }
    }
    // in-order wrap: pieces of a quarter go round the ring many times
    {
        ReqRing ring(1024);
        std::vector<uint64_t> q;
        for (int i = 0; i < 100; ++i, ++step) {
            uint64_t at = 0;
            if (q.size() == 4) {
                ring.give(q.front());
                q.erase(q.begin());
            }
            if (!ring.take(256, &at)) return fail("quarter refused with a quarter free", step);
            if (at != (uint64_t)(i % 4) * 256) return fail("wrap order", step);
            q.push_back(at);
        }
        uint64_t at = 0;
        if (ring.take(1, &at)) return fail("took from a full ring", step);
        // a piece given back out of order frees nothing until the oldest is back
        ring.give(q[2]);
        if (ring.take(256, &at)) return fail("reused a range behind the tail", step);
        ring.give(q[0]);
        if (!ring.take(256, &at) || at != q[0]) return fail("oldest range not reused", step);
    }
    // bad input
    {
        ReqRing ring(1024);
        uint64_t at = 0;
        if (ring.take(0, &at) || ring.take(1025, &at)) return fail("accepted a bad size", step);
        ring.give(12345);  // unknown offset: ignored
        if (!ring.take(1024, &at)) return fail("unknown give broke the ring", step);
    }
    std::printf("ok\n");
    return 0;
}
