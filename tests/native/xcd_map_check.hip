// Host check of the blend kernels' block -> tile mapping (blend_common.hpp):
// for random mixes of view sizes it must be a bijection on [0, total tiles),
// walk every XCD's share of a view contiguously, and reach the views in order
// of increasing tile count; xcd_of_tile must invert it; and the backward's
// balanced rank -> block deal (order_block, per XCD) must be a bijection.  Prints "ok" or
// the first failure; exit code 0/1.
#include <cstdio>
#include <random>
#include <vector>

#include "blend_common.hpp"

int main() {
  std::mt19937 rng(7);
  for (int trial = 0; trial < 2000; ++trial) {
    gsk::Views V{};
    V.n_views = 1 + int(rng() % GS_MAX_VIEWS);
    V.tile = 16;
    int total = 0;
    for (int k = 0; k < V.n_views; ++k) {
      V.v[k].gw = 1 + int(rng() % (trial % 3 == 0 ? 4 : 120));
      V.v[k].gh = 1 + int(rng() % (trial % 3 == 0 ? 3 : 80));
      V.v[k].W = V.v[k].gw * 16;
      V.v[k].H = V.v[k].gh * 16;
      V.v[k].tile_base = total;
      total += V.v[k].gw * V.v[k].gh;
    }
    V.total_tiles = total;
    const gsk::RViews R = gsk::make_rviews(V);
    std::vector<int> seen(total, 0);
    std::vector<int> first_block(V.n_views, -1);
    for (int b = 0; b < total; ++b) {
      const int t = gsk::xcd_tile(b, R);
      if (t < 0 || t >= total || seen[t]++) {
        std::printf("trial %d: block %d -> tile %d (total %d) repeated or out of range\n", trial,
                    b, t, total);
        return 1;
      }
      int idx = -1;
      const int x = gsk::xcd_of_tile(t, R, idx);
      if (x != b % gsk::kXcds || idx != b / gsk::kXcds) {
        std::printf("trial %d: tile %d of block %d maps back to XCD %d index %d\n", trial, t, b,
                    x, idx);
        return 1;
      }
      int v = 0;
      for (int k = 1; k < V.n_views; ++k) v = (V.v[k].tile_base <= t) ? k : v;
      if (first_block[v] < 0) first_block[v] = b;
    }
    // the backward's balanced order: each XCD's ranks dealt to its own blocks
    // cover every block exactly once
    std::vector<int> hit(total, 0);
    for (int x = 0; x < gsk::kXcds; ++x) {
      const int n_x = R.xcd_off[x][V.n_views];
      for (int r = 0; r < n_x; ++r) {
        const int b = gsk::order_block(r, n_x) * gsk::kXcds + x;
        if (b < 0 || b >= total || hit[b]++) {
          std::printf("trial %d: XCD %d rank %d -> block %d repeated or out of range\n", trial,
                      x, r, b);
          return 1;
        }
      }
    }
    // a view with fewer tiles never starts after a view with more tiles
    for (int a = 0; a < V.n_views; ++a)
      for (int c = 0; c < V.n_views; ++c) {
        const int ta = V.v[a].gw * V.v[a].gh, tc = V.v[c].gw * V.v[c].gh;
        if (ta < tc && first_block[a] > first_block[c]) {
          std::printf("trial %d: view %d (%d tiles) starts after view %d (%d tiles)\n", trial, a,
                      ta, c, tc);
          return 1;
        }
      }
  }
  // the backward's balanced order: ranks -> blocks is a bijection for any
  // tile count, pairs rank r of an odd complete round with block
  // round * kOrderRound + (kOrderRound - 1 - j), and keeps the last partial round
  for (int trial = 0; trial < 4000; ++trial) {
    const int n = trial < 2100 ? trial : 1 + int(rng() % 200000);
    std::vector<int> seen(n, 0);
    for (int r = 0; r < n; ++r) {
      const int b = gsk::order_block(r, n, gsk::kOrderRound);
      if (b < 0 || b >= n || seen[b]++) {
        std::printf("order n=%d: rank %d -> block %d repeated or out of range\n", n, r, b);
        return 1;
      }
      const int round = r / gsk::kOrderRound;
      const bool rev = (round & 1) && (round + 1) * gsk::kOrderRound <= n;
      if ((b / gsk::kOrderRound != round) || (rev != (b != r))) {
        std::printf("order n=%d: rank %d -> block %d outside its round\n", n, r, b);
        return 1;
      }
    }
  }
  std::printf("ok\n");
  return 0;
}
