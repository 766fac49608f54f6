#include "plan_logic.h"

#include <algorithm>

namespace dg {

std::vector<Tile> build_tiles(int64_t n_sub, const int64_t* off, int nb, uint16_t problem) {
    std::vector<Tile> tiles;
    int64_t n = 0;
    for (int64_t s = 0; s < n_sub; ++s) n += (off[s + 1] - off[s] + nb - 1) / nb;
    tiles.reserve((size_t)n);
    for (int64_t s = 0; s < n_sub; ++s)
        for (int64_t b = off[s]; b < off[s + 1]; b += nb) {
            Tile t;
            t.begin = b;
            t.sub = (int32_t)s;
            t.count = (uint16_t)std::min<int64_t>(nb, off[s + 1] - b);
            t.problem = problem;
            tiles.push_back(t);
        }
    return tiles;
}

std::vector<Tile> build_tiles_fitted(int64_t n_sub, const int64_t* off, const uint32_t* start, int nb,
                                     int support, int64_t cap_cells, int min_fit, uint16_t problem, int pad_to) {
    std::vector<Tile> tiles;
    for (int64_t s = 0; s < n_sub; ++s) {
        int64_t i = off[s];
        const int64_t e = off[s + 1];
        while (i < e) {
            // longest prefix (at most nb) whose box fits
            int32_t xl = 0, xh = -1, yl = 0, yh = -1;   // empty box
            int64_t k = 0;
            while (k < nb && i + k < e) {
                const uint32_t st = start[i + k];
                if (st != kNoStart) {
                    const int32_t x = (int32_t)(st & 0xFFFFu), y = (int32_t)(st >> 16);
                    const int32_t nxl = xh < xl ? x : std::min(xl, x), nxh = xh < xl ? x : std::max(xh, x);
                    const int32_t nyl = yh < yl ? y : std::min(yl, y), nyh = yh < yl ? y : std::max(yh, y);
                    const int64_t w = nxh - nxl + support;
                    const int64_t area = (w + (pad_to ? ((pad_to / 2 - w) & (pad_to - 1)) : 0)) * (nyh - nyl + support);
                    if (area > cap_cells) break;
                    xl = nxl; xh = nxh; yl = nyl; yh = nyh;
                }
                ++k;
            }
            int64_t n = k;
            if (k < min_fit && i + k < e) n = std::min<int64_t>(nb, e - i);
            if (n < 1) n = 1;
            Tile t;
            t.begin = i;
            t.sub = (int32_t)s;
            t.count = (uint16_t)n;
            t.problem = problem;
            tiles.push_back(t);
            i += n;
        }
    }
    return tiles;
}

BlockLists build_block_lists(int64_t n_sub, const int64_t* off, const uint32_t* vis_of, const uint32_t* start,
                             int n_v, int n_u, int block, int support) {
    const int nby = n_v / block, nbx = n_u / block;
    const int64_t n_blocks = n_sub * nby * nbx;
    BlockLists bl;
    bl.offsets.assign((size_t)n_blocks + 1, 0);
    // blocks overlapped by the neighbourhood that starts at (x0, y0)
    auto span = [&](int c0, int nb, int& lo, int& hi) {
        lo = std::max(0, c0 / block);
        hi = std::min(nb - 1, (c0 + support - 1) / block);
    };
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<int64_t> fill;
        if (pass == 1) {
            for (int64_t b = 0; b < n_blocks; ++b) bl.offsets[b + 1] += bl.offsets[b];
            bl.items.resize((size_t)bl.offsets[n_blocks]);
            fill.assign(bl.offsets.begin(), bl.offsets.end() - 1);
        }
        for (int64_t s = 0; s < n_sub; ++s)
            for (int64_t p = off[s]; p < off[s + 1]; ++p) {
                const uint32_t st = start[p];
                if (st == kNoStart) continue;
                const int x0 = (int)(st & 0xFFFFu), y0 = (int)(st >> 16);
                int bx_lo, bx_hi, by_lo, by_hi;
                span(x0, nbx, bx_lo, bx_hi);
                span(y0, nby, by_lo, by_hi);
                for (int by = by_lo; by <= by_hi; ++by)
                    for (int bx = bx_lo; bx <= bx_hi; ++bx) {
                        const int64_t b = (s * nby + by) * nbx + bx;
                        if (pass == 0) bl.offsets[b + 1]++;
                        else bl.items[(size_t)fill[b]++] = vis_of[p];
                    }
            }
    }
    return bl;
}

QueueSpec split_queues_weighted(const std::vector<int64_t>& weights) {
    QueueSpec q{};
    const int64_t n = (int64_t)weights.size();
    const int nq = (int)std::min<int64_t>(kMaxQueues, std::max<int64_t>(1, n));
    q.n_queues = nq;
    int64_t total = 0;
    for (int64_t w : weights) total += w;
    int64_t acc = 0;
    int cur = 0;
    q.begin[0] = 0;
    for (int64_t i = 0; i < n && cur < nq - 1; ++i) {
        acc += weights[(size_t)i];
        // close queue 'cur' once it holds its share of the weight
        if (acc * nq >= total * (int64_t)(cur + 1)) {
            q.end[cur] = (int32_t)(i + 1);
            ++cur;
            q.begin[cur] = (int32_t)(i + 1);
        }
    }
    for (int c = cur; c < nq; ++c) {
        if (c > cur) q.begin[c] = (int32_t)n;
        q.end[c] = (int32_t)n;
    }
    return q;
}

StaticDeal deal_static(const QueueSpec& q, int blocks, int waves_per_block) {
    StaticDeal d{};
    const int nq = q.n_queues;
    // every queue holds at most one tile per serving wavefront: all dealt
    // statically, no cursor and no stealing
    bool small = nq > 0;
    for (int k = 0; k < nq; ++k) {
        const int nb = blocks > k ? (blocks - k + nq - 1) / nq : 0;
        small = small && nb > 0 && (int64_t)q.end[k] - q.begin[k] <= (int64_t)nb * waves_per_block;
    }
    if (small) {
        for (int k = 0; k < nq; ++k) {
            d.sbase[k] = q.end[k];
            d.stride[k] = ((blocks - k + nq - 1) / nq) * waves_per_block;
        }
        d.on = 1;
        d.all_static = 1;
        return d;
    }
    for (int k = 0; k < kMaxQueues; ++k) {
        if (k >= nq) continue;
        const int nb = blocks > k ? (blocks - k + nq - 1) / nq : 0;
        const int w = nb * waves_per_block;
        const int64_t size = (int64_t)q.end[k] - q.begin[k];
        const int64_t base = (nb > 0 && size >= (int64_t)kMinTilesPerWave * w) ? size * kStaticEighths / 8 : 0;
        d.sbase[k] = q.begin[k] + (int32_t)base;
        d.stride[k] = w;
        if (base > 0) d.on = 1;
    }
    return d;
}

QueueSpec split_queues(const std::vector<Tile>& tiles) {
    std::vector<int64_t> w(tiles.size());
    for (size_t i = 0; i < tiles.size(); ++i) w[i] = tiles[i].count;
    return split_queues_weighted(w);
}

}  // namespace dg
