// CPU check of the device sub-allocator's logic (csrc/suballoc.h) over a
// malloc backend: random allocations and frees, blocks written and checked
// for overlap, the structure's invariants after every step, trims.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "suballoc.h"

struct MallocBackend {
    size_t *live;
    size_t round(size_t n) const { return (n + 4095) / 4096 * 4096; }
    void *allocate(size_t n) {
        if (*live + n > (size_t(3) << 30)) return nullptr;  // a 3 GiB "device"
        void *p = std::aligned_alloc(256, n);  // device segments are 256-byte aligned
        if (p) *live += n;
        return p;
    }
    void release(void *p, size_t n) {
        std::free(p);
        *live -= n;
    }
};

int main() {
    size_t live = 0;
    spc::SubAlloc<MallocBackend> sa(MallocBackend{&live});
    std::mt19937_64 rng(11);
    struct Held {
        unsigned char *p;
        size_t n;
        unsigned char tag;
    };
    std::vector<Held> held;
    long fails = 0, steps = 0;
    for (int it = 0; it < 60000; it++) {
        const int op = (int)(rng() % 10);
        if (op < 5 || held.empty()) {
            size_t n;
            switch (rng() % 4) {
                case 0: n = rng() % 4096; break;
                case 1: n = rng() % (size_t(2) << 20); break;
                case 2: n = rng() % (size_t(64) << 20); break;
                default: n = rng() % (size_t(300) << 20); break;
            }
            size_t got = 0;
            void *p = sa.alloc(n, &got);
            if (!p) {
                fails++;
                continue;
            }
            if (got < n || reinterpret_cast<uintptr_t>(p) % 256) {
                std::printf("bad block: asked %zu got %zu at %p\n", n, got, p);
                return 1;
            }
            const unsigned char tag = (unsigned char)(rng() % 251 + 1);
            const size_t touch = n < 64 ? n : 64;  // first and last bytes carry the tag
            std::memset(p, tag, touch);
            if (n > touch) std::memset(static_cast<unsigned char *>(p) + n - touch, tag, touch);
            held.push_back({static_cast<unsigned char *>(p), n, tag});
        } else if (op < 9) {
            const size_t k = rng() % held.size();
            const Held h = held[k];
            const size_t touch = h.n < 64 ? h.n : 64;
            for (size_t i = 0; i < touch; i++)
                if (h.p[i] != h.tag || (h.n > touch && h.p[h.n - 1 - i] != h.tag)) {
                    std::printf("overwritten block at %p (size %zu)\n", (void *)h.p, h.n);
                    return 1;
                }
            if (!sa.release(h.p)) {
                std::printf("release refused\n");
                return 1;
            }
            if (sa.release(h.p)) {
                std::printf("double release accepted\n");
                return 1;
            }
            held[k] = held.back();
            held.pop_back();
        } else {
            const size_t before = sa.segment_bytes();
            const size_t back = sa.trim(rng() % (size_t(512) << 20));
            if (sa.segment_bytes() != before - back) {
                std::printf("trim accounting\n");
                return 1;
            }
        }
        steps++;
        if (!sa.check()) {
            std::printf("invariants broken at step %d\n", it);
            return 1;
        }
        if (sa.segment_bytes() != live) {
            std::printf("segments %zu vs backend %zu\n", sa.segment_bytes(), live);
            return 1;
        }
    }
    for (auto &h : held) sa.release(h.p);
    if (!sa.check() || sa.used_bytes() != 0) {
        std::printf("not empty after freeing all\n");
        return 1;
    }
    sa.trim(0);
    if (sa.segments() != 0 || live != 0) {
        std::printf("segments left after trim(0): %zu\n", sa.segments());
        return 1;
    }
    std::printf("ok: %ld steps, %ld allocations refused by the backend\n", steps, fails);
    return 0;
}
