// Order of the block pairs of the symmetric product (host code, plain C++).
//
// The symmetric scheme evaluates every unordered pair of elements once: a
// tile is a pair of blocks of 256 elements (I, J), I <= J, whose (i, j) terms
// go to the rows of block I and whose (j, i) terms go to the rows of block J.
// The tiles are listed in rounds of a round-robin tournament (the circle
// method): in every round each block takes part in exactly one tile, so the
// tiles of one round write disjoint rows and can share one partial-sum slot
// per row.  With nbk blocks there are nbk rounds:
//   * nbk odd: a dummy block D = nbk completes an even field; the blocks
//     0 .. nbk-1 rotate around it.  In round r block r meets D, which stands
//     for its diagonal tile (r, r); the other blocks pair up as
//     ((r + k) mod nbk, (r - k) mod nbk), k = 1 .. (nbk - 1)/2.
//   * nbk even: block nbk - 1 stays fixed and the others rotate: round r
//     (0 <= r < nbk - 1) pairs r with nbk - 1 and ((r + k) mod (nbk - 1),
//     (r - k) mod (nbk - 1)), k = 1 .. nbk/2 - 1; the last round holds all
//     the diagonal tiles (K, K).
// Every unordered pair of distinct blocks meets in exactly one round (the
// property of the circle method), and every block has its diagonal tile in
// exactly one round.
//
// A product keeps at most S slots of partial sums per row (S from the
// partial-sum budget): rounds are taken in passes of S consecutive rounds,
// round r of a pass writing slot r mod S, and the slots of a pass are folded
// into an FP64 accumulator in slot order before the next pass reuses them.
#pragma once
#include <utility>
#include <vector>

namespace gabi {

// Calls f(I, J), I <= J, for every tile of round r (0 <= r < nbk) of nbk
// blocks.
template <typename F>
inline void sym_round_each(int nbk, int r, F &&f) {
    auto add = [&](int a, int b) { f(a < b ? a : b, a < b ? b : a); };
    if (nbk % 2 == 1) {
        const int M = nbk;  // rotating blocks 0 .. nbk-1 around the dummy
        add(r, r);
        for (int k = 1; k <= (nbk - 1) / 2; ++k) add((r + k) % M, (r - k + M) % M);
        return;
    }
    if (r == nbk - 1) {  // the diagonal round
        for (int K = 0; K < nbk; ++K) add(K, K);
        return;
    }
    const int M = nbk - 1;  // rotating blocks 0 .. nbk-2 around block nbk-1
    add(r, nbk - 1);
    for (int k = 1; k <= nbk / 2 - 1; ++k) add((r + k) % M, (r - k + M) % M);
}

// The tiles of round r as a list.
inline void sym_round(int nbk, int r, std::vector<std::pair<int, int>> &out) {
    out.clear();
    sym_round_each(nbk, r, [&](int a, int b) { out.emplace_back(a, b); });
}

// Most passes a product may take: more passes than this take more slots.
constexpr int kMaxPasses = 1024;

// Passes and slots of a symmetric product of nbk blocks when at most
// max_slots partial-sum slots per row fit: passes = ceil(nbk / max_slots),
// slots = ceil(nbk / passes) rounds per pass (the last pass may have fewer).
inline void sym_passes(int nbk, long long max_slots, int &passes, int &slots) {
    if (nbk < 1) {
        passes = slots = 1;
        return;
    }
    if (max_slots < 1) max_slots = 1;
    const long long min_slots = (nbk + kMaxPasses - 1) / kMaxPasses;
    if (max_slots < min_slots) max_slots = min_slots;
    passes = (int)((nbk + max_slots - 1) / max_slots);
    slots = (nbk + passes - 1) / passes;
    passes = (nbk + slots - 1) / slots;  // every pass non-empty
}

}  // namespace gabi
