// Map from a request id (the caller's 64-bit rid) to a pointer, for the
// request loop's finished-but-unreleased requests (host only).
//
// Open addressing with linear probing in a power-of-two table kept at most
// half full; ids are spread by the SplitMix64 output function (S. Vigna's
// published mixer), so sequential ids do not cluster. Removal shifts later
// entries of the same probe run back (no tombstones), so lookups stay short
// under a steady insert/remove load. A null pointer marks an empty slot, so
// stored pointers must be non-null. Not thread-safe.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace mtgp_impl {

template <class T>
class RidMap {
public:
    RidMap() : slots_(64) {}

    size_t size() const { return count_; }

    // Map rid to p (p non-null); replaces an existing entry for rid.
    void put(uint64_t rid, T *p)
    {
        if (2 * (count_ + 1) > slots_.size())
            grow();
        size_t i = home(rid);
        while (slots_[i].p) {
            if (slots_[i].rid == rid) {
                slots_[i].p = p;
                return;
            }
            i = (i + 1) & mask();
        }
        slots_[i] = Slot{rid, p};
        count_++;
    }

    // Remove rid's entry and return its pointer (nullptr if absent).
    T *take(uint64_t rid)
    {
        size_t i = home(rid);
        while (slots_[i].p) {
            if (slots_[i].rid == rid) {
                T *p = slots_[i].p;
                erase_at(i);
                return p;
            }
            i = (i + 1) & mask();
        }
        return nullptr;
    }

    template <class F>
    void for_each(F f) const
    {
        for (const Slot &s : slots_)
            if (s.p)
                f(s.rid, s.p);
    }

private:
    struct Slot {
        uint64_t rid = 0;
        T *p = nullptr;
    };
    std::vector<Slot> slots_;
    size_t count_ = 0;

    size_t mask() const { return slots_.size() - 1; }

    size_t home(uint64_t rid) const
    {
        uint64_t z = rid + 0x9e3779b97f4a7c15ull;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return (size_t)(z ^ (z >> 31)) & mask();
    }

    // Empty slot i, then move back every later entry of the run whose home
    // does not lie cyclically in (i, j], so that no lookup meets a gap before
    // its entry.
    void erase_at(size_t i)
    {
        size_t j = i;
        for (;;) {
            j = (j + 1) & mask();
            if (!slots_[j].p)
                break;
            const size_t h = home(slots_[j].rid);
            const bool stays = i <= j ? (i < h && h <= j) : (i < h || h <= j);
            if (!stays) {
                slots_[i] = slots_[j];
                i = j;
            }
        }
        slots_[i] = Slot{};
        count_--;
    }

    void grow()
    {
        std::vector<Slot> old(slots_.size() * 2);
        old.swap(slots_);
        count_ = 0;
        for (const Slot &s : old)
            if (s.p)
                put(s.rid, s.p);
    }
};

}  // namespace mtgp_impl
