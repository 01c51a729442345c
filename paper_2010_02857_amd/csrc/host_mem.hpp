// Host memory for the plan's large tables.
#pragma once

#include <cstddef>
#include <vector>

namespace ifgf {

// Has the kernel map the pages of [p, p + bytes) on the plan builder's thread
// pool (MADV_POPULATE_WRITE, in huge pages where the system grants them).
// Filling gigabytes of fresh memory from one thread pays one page fault per
// 4 KiB and was the largest host cost of the frame and tile tables.  Blocks
// under 16 MiB are left alone; a kernel without the call leaves the pages to
// fault in when they are first written, as without it.
void map_pages(void* p, size_t bytes);

// Empties v and reserves room for n elements over mapped pages; the caller
// still fills v (assign, resize or a copy).
template <class T>
void reserve_mapped(std::vector<T>& v, size_t n)
{
    std::vector<T>().swap(v);
    v.reserve(n);
    map_pages(v.data(), n * sizeof(T));
}

}  // namespace ifgf
