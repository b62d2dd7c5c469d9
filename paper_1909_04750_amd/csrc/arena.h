// Host-side allocator of the server's output budget (plain C++, no device code).
#pragma once
#include <algorithm>
#include <cstddef>
#include <map>
#include <utility>
#include <vector>

namespace serve_arena {

// Output-arena allocator, in 32-bit words.  A request is rounded up to a size class with
// three significant bits (exact up to 8 words, then steps of 1/8 of a power of two, so at
// most 12.5% of a block is unused); each class keeps a stack of free blocks, and new blocks
// are cut from the top of the arena.  When neither serves, a first-fit list of spare
// blocks is tried, then every free block is merged with its neighbours into that list
// (and the top lowered when the highest free block reaches it) and the allocation is
// retried; a block of a larger class is split only after that.  Alloc
// and release are O(1) in the steady state.
struct Arena {
    size_t capacity = 0, top = 0;
    size_t listed = 0;                            // words in the class stacks
    std::vector<std::vector<size_t>> lists;       // per class: block offsets
    std::map<size_t, size_t> spare;               // merged free blocks: offset -> words
    size_t spare_words = 0;
    bool released_since_merge = false;            // a merge can only help after a release

    static int cls(size_t w)
    {
        if (w <= 8) return (int)w - 1;
        int e = 63 - __builtin_clzll((unsigned long long)w);  // 2^e <= w < 2^(e+1), e >= 3
        size_t m = (w + ((size_t)1 << (e - 3)) - 1) >> (e - 3);  // ceil(w / 2^(e-3)) in 8..16
        if (m == 16) {
            e++;
            m = 8;
        }
        return 8 + (e - 3) * 8 + (int)(m - 8);
    }
    static size_t class_words(int c) { return c < 8 ? (size_t)c + 1 : (size_t)(8 + (c - 8) % 8) << ((c - 8) / 8); }

    void reset(size_t words)
    {
        capacity = words;
        top = 0;
        listed = 0;
        lists.assign(cls(words) + 2, {});
        spare.clear();
        spare_words = 0;
        released_since_merge = false;
    }
    bool from_spare(size_t need, size_t *off)
    {
        for (auto it = spare.begin(); it != spare.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const size_t rest = it->second - need, start = it->first + need;
                spare.erase(it);
                if (rest) spare[start] = rest;
                spare_words -= need;
                return true;
            }
        }
        return false;
    }
    // Merge every listed and spare block, and give a free block at the top back to it.
    void merge_all()
    {
        std::vector<std::pair<size_t, size_t>> blocks(spare.begin(), spare.end());
        for (size_t c = 0; c < lists.size(); c++)
            for (size_t o : lists[c]) blocks.emplace_back(o, class_words((int)c));
        for (auto &l : lists) l.clear();
        listed = 0;
        spare.clear();
        spare_words = 0;
        released_since_merge = false;
        std::sort(blocks.begin(), blocks.end());
        for (size_t i = 0; i < blocks.size();) {
            size_t o = blocks[i].first, w = blocks[i].second;
            for (i++; i < blocks.size() && blocks[i].first == o + w; i++) w += blocks[i].second;
            if (o + w == top) {
                top = o;
            } else {
                spare[o] = w;
                spare_words += w;
            }
        }
    }
    // On success *granted is the block size to pass back to release().  Order: a block of
    // the exact class, the top, a spare block (first fit, low offsets first); failing
    // those, merge all free space and try again; splitting a larger class's block comes
    // last, because merging keeps the free space in fewer, larger pieces.
    bool alloc(size_t words, size_t *off, size_t *granted)
    {
        const int c = cls(words);
        const size_t need = class_words(c);
        *granted = need;
        for (int pass = 0; pass < 2; pass++) {
            if (!lists[c].empty()) {
                *off = lists[c].back();
                lists[c].pop_back();
                listed -= need;
                return true;
            }
            if (top + need <= capacity) {
                *off = top;
                top += need;
                return true;
            }
            if (spare_words >= need && from_spare(need, off)) return true;
            if (pass == 0 && released_since_merge && listed + spare_words >= need) merge_all();
            else break;
        }
        for (size_t b = c + 1; b < lists.size(); b++) {
            if (!lists[b].empty()) {  // split a block of a larger class
                *off = lists[b].back();
                lists[b].pop_back();
                const size_t bw = class_words((int)b);
                listed -= bw;
                spare[*off + need] = bw - need;
                spare_words += bw - need;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t granted)
    {
        lists[cls(granted)].push_back(off);
        listed += granted;
        released_since_merge = true;
    }
    size_t free_words() const
    {
        return capacity - top + listed + spare_words;
    }
};

}  // namespace serve_arena
