// Index of the free ranges of the request loop's output arena (host only).
//
// Two-level segregated fit (M. Masmano et al., "TLSF: a new dynamic memory
// allocator for real-time systems", 2004), over units of the arena's
// alignment: free blocks sit in size classes -- a power-of-two range split
// into 16 equal parts, exact sizes below 16 units -- with one bit per
// non-empty class, so finding a class whose every block is large enough is
// two bit scans. Blocks keep links to their physical neighbours, so a released
// block merges with free neighbours in O(1). A take first looks in the classes
// above the request's own (good fit), then scans the request's own class for a
// block that is large enough, so it fails only when no free block can hold the
// request. Not thread-safe.
#pragma once

#include <stdint.h>

#include <vector>

namespace mtgp_impl {

class ArenaIndex {
public:
    static constexpr uint32_t kNil = UINT32_MAX;

    // `units` units of the arena, one free block
    explicit ArenaIndex(uint64_t units)
    {
        for (auto &row : heads_)
            for (uint32_t &h : row)
                h = kNil;
        if (units > 0)
            insert(make_block(0, units, kNil, kNil));
    }

    // A block of `units` units (> 0): its id, or kNil if no free block is
    // large enough. offset(id) gives its start.
    uint32_t take(uint64_t units)
    {
        uint32_t id = find_above(units);
        if (id == kNil)
            id = find_in_class(units);
        if (id == kNil)
            return kNil;
        unlink(id);
        Block &b = blocks_[id];
        if (b.len > units) {
            const uint32_t rest = make_block(b.off + units, b.len - units, id, b.next_phys);
            Block &bb = blocks_[id];   // make_block may have moved the vector
            if (bb.next_phys != kNil)
                blocks_[bb.next_phys].prev_phys = rest;
            bb.next_phys = rest;
            bb.len = units;
            insert(rest);
        }
        blocks_[id].free = false;
        return id;
    }

    // Return a block from take().
    void give(uint32_t id)
    {
        Block *b = &blocks_[id];
        b->free = true;
        const uint32_t nx = b->next_phys;
        if (nx != kNil && blocks_[nx].free) {
            unlink(nx);
            b->len += blocks_[nx].len;
            b->next_phys = blocks_[nx].next_phys;
            if (b->next_phys != kNil)
                blocks_[b->next_phys].prev_phys = id;
            spare_.push_back(nx);
        }
        const uint32_t pv = b->prev_phys;
        if (pv != kNil && blocks_[pv].free) {
            unlink(pv);
            Block &p = blocks_[pv];
            p.len += b->len;
            p.next_phys = b->next_phys;
            if (p.next_phys != kNil)
                blocks_[p.next_phys].prev_phys = pv;
            spare_.push_back(id);
            id = pv;
        }
        insert(id);
    }

    uint64_t offset(uint32_t id) const { return blocks_[id].off; }
    uint64_t length(uint32_t id) const { return blocks_[id].len; }

    // Free blocks as (offset, length), for checks.
    std::vector<std::pair<uint64_t, uint64_t>> free_blocks() const
    {
        std::vector<std::pair<uint64_t, uint64_t>> v;
        for (const auto &row : heads_)
            for (uint32_t h : row)
                for (uint32_t i = h; i != kNil; i = blocks_[i].next_free)
                    v.emplace_back(blocks_[i].off, blocks_[i].len);
        return v;
    }

private:
    struct Block {
        uint64_t off, len;
        uint32_t prev_phys, next_phys;   // physical neighbours (kNil: none)
        uint32_t prev_free, next_free;   // the class's free list
        bool free;
    };
    static constexpr int kFl = 64, kSl = 16;

    std::vector<Block> blocks_;
    std::vector<uint32_t> spare_;   // ids of merged-away blocks, for reuse
    uint64_t fl_map_ = 0;
    uint32_t sl_map_[kFl] = {};
    uint32_t heads_[kFl][kSl];

    static int log2_floor(uint64_t v) { return 63 - __builtin_clzll(v); }

    // class of a block of `units` units: exact below 16, else the power of
    // two and the sixteenth within it
    static void mapping(uint64_t units, int &fl, int &sl)
    {
        if (units < kSl) {
            fl = 0;
            sl = (int)units;
            return;
        }
        const int b = log2_floor(units);
        fl = b - 3;
        sl = (int)((units >> (b - 4)) - kSl);
    }

    uint32_t make_block(uint64_t off, uint64_t len, uint32_t prev_phys, uint32_t next_phys)
    {
        const Block b{off, len, prev_phys, next_phys, kNil, kNil, true};
        if (!spare_.empty()) {
            const uint32_t id = spare_.back();
            spare_.pop_back();
            blocks_[id] = b;
            return id;
        }
        blocks_.push_back(b);
        return (uint32_t)(blocks_.size() - 1);
    }

    void insert(uint32_t id)
    {
        Block &b = blocks_[id];
        b.free = true;
        int fl, sl;
        mapping(b.len, fl, sl);
        b.prev_free = kNil;
        b.next_free = heads_[fl][sl];
        if (b.next_free != kNil)
            blocks_[b.next_free].prev_free = id;
        heads_[fl][sl] = id;
        fl_map_ |= 1ull << fl;
        sl_map_[fl] |= 1u << sl;
    }

    void unlink(uint32_t id)
    {
        Block &b = blocks_[id];
        int fl, sl;
        mapping(b.len, fl, sl);
        if (b.prev_free != kNil)
            blocks_[b.prev_free].next_free = b.next_free;
        else
            heads_[fl][sl] = b.next_free;
        if (b.next_free != kNil)
            blocks_[b.next_free].prev_free = b.prev_free;
        if (heads_[fl][sl] == kNil) {
            sl_map_[fl] &= ~(1u << sl);
            if (!sl_map_[fl])
                fl_map_ &= ~(1ull << fl);
        }
    }

    // first block of the first non-empty class whose every block holds
    // `units`: the class of units rounded up to the next class boundary
    uint32_t find_above(uint64_t units) const
    {
        uint64_t r = units;
        if (units >= kSl) {
            const int b = log2_floor(units);
            r = units + ((1ull << (b - 4)) - 1);
        }
        int fl, sl;
        mapping(r, fl, sl);
        if (fl >= kFl)
            return kNil;
        uint32_t sls = sl_map_[fl] & (~0u << sl);
        if (!sls) {
            const uint64_t fls = fl + 1 < kFl ? fl_map_ & (~0ull << (fl + 1)) : 0;
            if (!fls)
                return kNil;
            fl = __builtin_ctzll(fls);
            sls = sl_map_[fl];
        }
        return heads_[fl][__builtin_ctz(sls)];
    }

    // a block of the request's own class that holds it (the class's blocks
    // span a range of sizes)
    uint32_t find_in_class(uint64_t units) const
    {
        int fl, sl;
        mapping(units, fl, sl);
        for (uint32_t i = heads_[fl][sl]; i != kNil; i = blocks_[i].next_free)
            if (blocks_[i].len >= units)
                return i;
        return kNil;
    }
};

}  // namespace mtgp_impl
