// Sub-allocation of large device segments: best fit over the free blocks of
// every segment, a block split when the rest is worth keeping, neighbours
// coalesced when freed, and whole free segments returned on trim.  Host code
// with no HIP call of its own: the backend (segment size rounding, allocate,
// release) is a template parameter, so the same logic runs over malloc in a
// CPU test.  Not thread-safe: the caller serialises.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace spc {

template <typename Backend>
class SubAlloc {
  public:
    // requests are rounded to kAlign; a free remainder of at least kSplit
    // becomes a block of its own; segments are at least kMinSegment bytes
    static constexpr size_t kAlign = 256;
    static constexpr size_t kSplit = size_t(1) << 20;
    static constexpr size_t kMinSegment = size_t(64) << 20;

    explicit SubAlloc(Backend be = Backend()) : be_(be) {}
    SubAlloc(const SubAlloc &) = delete;
    SubAlloc &operator=(const SubAlloc &) = delete;

    // a block of at least `bytes` (*got = its size), or nullptr when the
    // backend has no new segment to give
    void *alloc(size_t bytes, size_t *got) {
        bytes = (bytes ? bytes + kAlign - 1 : kAlign) / kAlign * kAlign;
        auto f = free_.lower_bound(bytes);
        if (f == free_.end()) {
            const size_t seg = be_.round(bytes > kMinSegment ? bytes : kMinSegment);
            void *p = be_.allocate(seg);
            if (!p) return nullptr;
            const uintptr_t a = reinterpret_cast<uintptr_t>(p);
            segs_[a] = seg;
            blocks_[a] = Block{seg, a, true};
            f = free_.emplace(seg, a);
        }
        const uintptr_t a = f->second;
        free_.erase(f);
        Block &b = blocks_[a];
        if (b.size - bytes >= kSplit) {
            const uintptr_t r = a + bytes;
            blocks_[r] = Block{b.size - bytes, b.seg, true};
            free_.emplace(b.size - bytes, r);
            b.size = bytes;
        }
        b.free = false;
        used_ += b.size;
        *got = b.size;
        return reinterpret_cast<void *>(a);
    }

    // false if p is not a block of this allocator
    bool release(void *p) {
        auto it = blocks_.find(reinterpret_cast<uintptr_t>(p));
        if (it == blocks_.end() || it->second.free) return false;
        used_ -= it->second.size;
        it->second.free = true;
        // coalesce with the next and the previous block of the same segment
        auto nx = std::next(it);
        if (nx != blocks_.end() && nx->second.free && nx->second.seg == it->second.seg &&
            nx->first == it->first + it->second.size) {
            erase_free(nx->second.size, nx->first);
            it->second.size += nx->second.size;
            blocks_.erase(nx);
        }
        if (it != blocks_.begin()) {
            auto pv = std::prev(it);
            if (pv->second.free && pv->second.seg == it->second.seg &&
                pv->first + pv->second.size == it->first) {
                erase_free(pv->second.size, pv->first);
                pv->second.size += it->second.size;
                blocks_.erase(it);
                it = pv;
            }
        }
        free_.emplace(it->second.size, it->first);
        return true;
    }

    // give whole free segments back, largest first, until at most max_free
    // bytes of free blocks stay; returns the bytes given back
    size_t trim(size_t max_free) {
        size_t back = 0;
        for (auto f = free_.rbegin(); f != free_.rend() && free_bytes() > max_free;) {
            const uintptr_t a = f->second;
            const Block &b = blocks_[a];
            auto s = segs_.find(a);
            if (s != segs_.end() && s->second == b.size) {  // the segment is one free block
                const size_t sz = b.size;
                blocks_.erase(a);
                segs_.erase(s);
                f = decltype(f)(free_.erase(std::next(f).base()));
                be_.release(reinterpret_cast<void *>(a), sz);
                back += sz;
            } else {
                ++f;
            }
        }
        return back;
    }

    size_t free_bytes() const { return segment_bytes() - used_; }
    size_t used_bytes() const { return used_; }
    size_t segment_bytes() const {
        size_t t = 0;
        for (auto &s : segs_) t += s.second;
        return t;
    }
    size_t segments() const { return segs_.size(); }
    size_t blocks() const { return blocks_.size(); }
    bool owns(void *p) const { return blocks_.count(reinterpret_cast<uintptr_t>(p)) != 0; }
    // every block lies inside its segment, blocks tile each segment without
    // gap or overlap, no two free neighbours are left uncoalesced, and the
    // free index lists exactly the free blocks
    bool check() const {
        size_t nfree = 0, usedsum = 0;
        for (auto &s : segs_) {
            uintptr_t at = s.first;
            auto it = blocks_.find(s.first);
            bool prev_free = false;
            while (at < s.first + s.second) {
                if (it == blocks_.end() || it->first != at || it->second.seg != s.first) return false;
                if (it->second.free && prev_free) return false;
                prev_free = it->second.free;
                if (it->second.free)
                    nfree++;
                else
                    usedsum += it->second.size;
                at += it->second.size;
                ++it;
            }
            if (at != s.first + s.second) return false;
        }
        if (nfree != free_.size() || usedsum != used_) return false;
        for (auto &f : free_) {
            auto it = blocks_.find(f.second);
            if (it == blocks_.end() || !it->second.free || it->second.size != f.first) return false;
        }
        return true;
    }

  private:
    struct Block {
        size_t size;
        uintptr_t seg;  // base of the segment holding it
        bool free;
    };
    void erase_free(size_t size, uintptr_t a) {
        auto r = free_.equal_range(size);
        for (auto i = r.first; i != r.second; ++i)
            if (i->second == a) {
                free_.erase(i);
                return;
            }
    }
    Backend be_;
    std::map<uintptr_t, size_t> segs_;     // base -> size
    std::map<uintptr_t, Block> blocks_;    // address -> block
    std::multimap<size_t, uintptr_t> free_;  // size -> address of a free block
    size_t used_ = 0;
};

}  // namespace spc
