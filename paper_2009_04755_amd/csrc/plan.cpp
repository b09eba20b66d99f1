// Host planner: divide-and-conquer split of the pair matrix into tiles and the
// ordering of work items in the device queue.
//
// Section IV-B treats all pairs (i, j), i < j, as an upper-triangular matrix that is
// split into four quadrants recursively, skipping quadrants without work; the leaves
// are the jobs.  Here the recursion stops at blocks of T items, so every leaf is a
// tile of up to T x T pairs whose two item blocks are staged once in fast memory and
// reused T times each.  Leaves come out in recursion order (top-left, top-right,
// bottom-left, bottom-right): neighbouring leaves share item blocks, which is the
// locality the paper's workers get by preferring their own lowest-level tasks.
#include <algorithm>
#include <numeric>
#include <random>

#include "common.hpp"

namespace rk {

static bool quadrant_has_work(int64_t r0, int64_t r1, int64_t c0, int64_t c1, int64_t n)
{
    r1 = std::min(r1, n);
    c1 = std::min(c1, n);
    if (r0 >= r1 || c0 >= c1) return false;
    return std::max(c0, r0 + 1) <= c1 - 1;
}

static void rec(int64_t br, int64_t bc, int64_t size, int64_t T, int64_t n, std::vector<int2> &out)
{
    if (!quadrant_has_work(br * T, (br + size) * T, bc * T, (bc + size) * T, n)) return;
    if (size == 1) {
        out.push_back(make_int2((int)br, (int)bc));
        return;
    }
    const int64_t h = size / 2;
    rec(br, bc, h, T, n, out);
    rec(br, bc + h, h, T, n, out);
    rec(br + h, bc, h, T, n, out);
    rec(br + h, bc + h, h, T, n, out);
}

void plan_leaves(int64_t n, int64_t T, std::vector<int2> &out)
{
    out.clear();
    if (n < 2 || T < 1) return;
    const int64_t nb = (n + T - 1) / T;
    int64_t side = 1;
    while (side < nb) side *= 2;
    rec(0, 0, side, T, n, out);
}

// Work item = {bi, bj, chunk, tile index}.  Items are ordered chunk-major so that at any
// moment the whole chip works on a narrow window of the reduction dimension (its
// operands stay in the shared last-level cache); within a chunk the D&C leaf list is
// cut into nseg contiguous pieces, piece x feeding segment x (one per XCD), so that
// the workgroups of one XCD share item blocks through that XCD's L2.
// A tile may be processed as `halves` column slices (item .w = tile * halves + slice).
void plan_chunked(const std::vector<int2> &tiles, int nchunks, int nseg, std::vector<int4> &items,
                  std::vector<int> &seg, int halves)
{
    const int64_t nt = (int64_t)tiles.size() * halves;
    items.clear();
    items.reserve((size_t)(nt * nchunks));
    seg.assign((size_t)nseg + 1, 0);
    for (int s = 0; s < nseg; ++s) {
        const int64_t t0 = nt * s / nseg, t1 = nt * (s + 1) / nseg;
        for (int c = 0; c < nchunks; ++c)
            for (int64_t t = t0; t < t1; ++t)
                items.push_back(make_int4(tiles[t / halves].x, tiles[t / halves].y, c, (int)t));
        seg[s + 1] = (int)items.size();
    }
}

// Largest estimated cost first (the paper's stealing of the largest task), dealt
// round-robin so every segment gets a similar mix.
void plan_lpt(const std::vector<int4> &items_in, const std::vector<double> &cost, int nseg, std::vector<int4> &items,
              std::vector<int> &seg)
{
    std::vector<int64_t> order(items_in.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
    std::vector<std::vector<int4>> per(nseg);
    for (size_t k = 0; k < order.size(); ++k) per[k % nseg].push_back(items_in[order[k]]);
    items.clear();
    seg.assign((size_t)nseg + 1, 0);
    for (int s = 0; s < nseg; ++s) {
        items.insert(items.end(), per[s].begin(), per[s].end());
        seg[s + 1] = (int)items.size();
    }
}

void shuffle_items(std::vector<int4> &items, std::vector<int> &seg, uint64_t seed)
{
    std::mt19937_64 g(seed);
    std::shuffle(items.begin(), items.end(), g);
    single_segment(seg, (int64_t)items.size());
}

void single_segment(std::vector<int> &seg, int64_t nitems)
{
    seg.assign(2, 0);
    seg[1] = (int)nitems;
}

}  // namespace rk

extern "C" int64_t rocket_plan_tiles(int64_t n, int64_t T, int32_t *bi, int32_t *bj, int64_t cap)
{
    if (n < 0 || T < 1 || cap < 0 || (cap > 0 && (!bi || !bj))) return ROCKET_E_INVALID;
    std::vector<int2> leaves;
    rk::plan_leaves(n, T, leaves);
    const int64_t m = std::min<int64_t>(cap, (int64_t)leaves.size());
    for (int64_t k = 0; k < m; ++k) {
        bi[k] = leaves[k].x;
        bj[k] = leaves[k].y;
    }
    return (int64_t)leaves.size();
}

extern "C" int64_t rocket_pair_index(int64_t i, int64_t j, int64_t n)
{
    return i * n - i * (i + 1) / 2 + (j - i - 1);
}
