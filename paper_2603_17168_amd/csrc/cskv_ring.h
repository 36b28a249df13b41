// Ring allocator of the serving loop's output arena (host code, no HIP dependency).
// Allocations are freed in the order they were made (requests finish in admission order).
// Nonzero allocations are laid out in order, wrapping to offset 0 when the end is reached; the
// live bytes are [tail, head) before a wrap and [tail, size) + [0, head) after one, where tail
// is the start of the oldest and head the end of the newest nonzero allocation.
#pragma once

#include <stddef.h>

#include <deque>
#include <utility>

namespace cskv {

struct Ring {
    size_t size = 0, head = 0, tail = 0, last = 0;  // last: start of the newest nonzero allocation
    size_t nonzero = 0;
    std::deque<std::pair<size_t, size_t>> live;  // (offset, bytes) in allocation order

    // offset of `bytes` free bytes, or false if they do not fit now
    bool alloc(size_t bytes, size_t* off) {
        if (bytes > size) return false;
        if (bytes == 0) {  // takes no space; keeps its place in the completion order
            live.push_back({0, 0});
            *off = 0;
            return true;
        }
        size_t pos;
        if (nonzero == 0) {
            pos = 0;
            tail = 0;
        } else if (tail <= last) {  // not wrapped: free are [head, size) and [0, tail)
            if (head + bytes <= size) pos = head;
            else if (bytes <= tail) pos = 0;
            else return false;
        } else {  // wrapped: free is [head, tail)
            if (head + bytes <= tail) pos = head;
            else return false;
        }
        live.push_back({pos, bytes});
        ++nonzero;
        last = pos;
        head = pos + bytes;
        *off = pos;
        return true;
    }

    // release the oldest allocation
    void free_front() {
        if (live.front().second) --nonzero;
        live.pop_front();
        if (nonzero == 0) {
            head = tail = last = 0;
            return;
        }
        for (const auto& e : live) {  // the oldest allocation that holds bytes
            if (e.second) {
                tail = e.first;
                break;
            }
        }
    }
};

}  // namespace cskv
