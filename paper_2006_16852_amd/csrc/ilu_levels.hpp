// ilu_levels.hpp -- dependency levels of the triangular factors on A's
// pattern, the schedule of the exact (level-by-level) triangular solves of
// the ILU-type preconditioner (Sec. 3.2).
//
// Row i of the lower factor depends on the rows of its strictly lower
// entries, row i of the upper factor on the rows of its strictly upper
// entries.  level(i) = 1 + the largest level of the rows it depends on (0
// with none), so every row of a level can be solved at once after the
// earlier levels.  Rows are listed level by level, ascending within a level
// (a stable counting sort): perm[ptr[l] .. ptr[l+1]) are the rows of level l.
//
// Host-only standard C++: also compiled by g++ in the CPU tests.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace mxl {

inline void ilu_levels_host(const std::vector<int> &rp, const std::vector<int> &col, bool lower,
                            std::vector<int> &perm, std::vector<int64_t> &ptr) {
    const int64_t n = (int64_t)rp.size() - 1;
    std::vector<int> lev((size_t)n, 0);
    int maxl = 0;
    for (int64_t s = 0; s < n; ++s) {
        const int64_t i = lower ? s : n - 1 - s;
        int l = 0;
        for (int q = rp[(size_t)i]; q < rp[(size_t)i + 1]; ++q) {
            const int k = col[(size_t)q];
            if ((lower && k < i) || (!lower && k > i)) l = std::max(l, lev[(size_t)k] + 1);
        }
        lev[(size_t)i] = l;
        maxl = std::max(maxl, l);
    }
    ptr.assign(n > 0 ? (size_t)maxl + 2 : 1, 0);
    for (int64_t i = 0; i < n; ++i) ptr[(size_t)lev[(size_t)i] + 1]++;
    for (size_t l = 1; l < ptr.size(); ++l) ptr[l] += ptr[l - 1];
    perm.assign((size_t)n, 0);
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) perm[(size_t)fill[(size_t)lev[(size_t)i]]++] = (int)i;
}

// The schedule's invariants, checked before any level launch is built on it:
// ptr runs from 0 to n without decreasing and every level is non-empty,
// perm is a permutation of 0..n-1, and every dependency of a row lies in an
// earlier level.  Returns false on any violation.
inline bool ilu_levels_valid(const std::vector<int> &rp, const std::vector<int> &col, bool lower,
                             const std::vector<int> &perm, const std::vector<int64_t> &ptr) {
    const int64_t n = (int64_t)rp.size() - 1;
    if (ptr.empty() || ptr.front() != 0 || ptr.back() != n || (int64_t)perm.size() != n) return false;
    for (size_t l = 0; l + 1 < ptr.size(); ++l)
        if (ptr[l + 1] <= ptr[l]) return false;
    std::vector<int> lev((size_t)n, -1);
    for (size_t l = 0; l + 1 < ptr.size(); ++l)
        for (int64_t q = ptr[l]; q < ptr[l + 1]; ++q) {
            const int i = perm[(size_t)q];
            if (i < 0 || i >= n || lev[(size_t)i] != -1) return false;
            lev[(size_t)i] = (int)l;
        }
    for (int64_t i = 0; i < n; ++i)
        for (int q = rp[(size_t)i]; q < rp[(size_t)i + 1]; ++q) {
            const int k = col[(size_t)q];
            if (((lower && k < i) || (!lower && k > i)) && lev[(size_t)k] >= lev[(size_t)i]) return false;
        }
    return true;
}

}  // namespace mxl
