// Host-side choice of the set a fused pass holds in its tile, shared by the
// two-level and the three-level schedulers.
//
// A pass scans the operations not yet placed in stream order and takes one
// when it commutes with every earlier operation left behind and its target
// lies in the tile set.  Which set to pick is the only freedom.  Filling it
// first come, first served spends tile places on the targets of operations
// that are blocked soon after; instead the set grows one member at a time
// by the candidate that lets the scan take the most operations of a window
// of the next ones, and then single exchanges of a chosen member for another
// candidate are made while each takes more.  Any set gives a valid pass, so
// this only decides how many operations each pass carries.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace qsim {

// One operation as the scan sees it: x = the members whose values it changes,
// z = the members it only reads (controls, conditions, diagonal targets),
// t = the member that must lie in the tile set (0 if none).  Two operations
// commute when neither one's x meets the other's x or z.
struct ScanOp {
    uint64_t x, z, t;
};

// Operations of w the scan takes with the fixed set S (at most cap).  The
// lookahead calls this a few thousand times per pass, so it is written
// without branches.
inline size_t scan_count(const std::vector<ScanOp> &w, uint64_t S, size_t cap)
{
    uint64_t bx = 0, bz = 0;
    size_t n = 0;
    for (const ScanOp &u : w) {
        const uint64_t blocked = (u.x & (bx | bz)) | (u.z & bx) | (u.t & ~S);
        const uint64_t take = (blocked == 0) & (n < cap);
        const uint64_t keep = take - 1;  // all ones when the operation stays behind
        n += take;
        bx |= u.x & keep;
        bz |= u.z & keep;
    }
    return n;
}

// The set for the next pass: S0 (always held) plus at most k - |S0| of the
// targets of w.
inline uint64_t lookahead_set(const std::vector<ScanOp> &w, uint64_t S0, int k, size_t cap,
                              int max_exchanges)
{
    uint64_t cand = 0;
    for (const ScanOp &u : w)
        cand |= u.t;
    cand &= ~S0;
    uint64_t S = S0;
    size_t best = scan_count(w, S, cap);
    while (__builtin_popcountll(S) < k && (cand & ~S) != 0) {
        uint64_t pick = 0;
        size_t pc = 0;
        for (uint64_t m = cand & ~S; m != 0; m &= m - 1) {
            const uint64_t b = m & (~m + 1);
            const size_t c = scan_count(w, S | b, cap);
            if (pick == 0 || c > pc) {
                pick = b;
                pc = c;
            }
        }
        S |= pick;
        best = pc;
    }
    for (int moves = 0; moves < max_exchanges; ++moves) {
        bool better = false;
        for (uint64_t a = S & ~S0; a != 0 && !better; a &= a - 1) {
            const uint64_t ba = a & (~a + 1);
            for (uint64_t m = cand & ~S; m != 0; m &= m - 1) {
                const uint64_t bb = m & (~m + 1);
                const uint64_t T = (S & ~ba) | bb;
                const size_t c = scan_count(w, T, cap);
                if (c > best) {
                    S = T;
                    best = c;
                    better = true;
                    break;
                }
            }
        }
        if (!better)
            break;
    }
    return S;
}

}  // namespace qsim
