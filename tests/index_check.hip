// index_check.hip -- host-side check of the fused tile kernels' indexing.
//
// Runs on the CPU, no device: for every tile shape, K = 1, 2 and 3 subcycles
// per pass and a set of domain sizes (ragged tails, one element wide, single
// element), it walks every tile, lane, element phase, node phase and node
// round the way k_fused / k_fused_multi do, computing each index with the
// kernels' own functions (mevp_index.hpp), and checks:
//   * every LDS read and write lies inside its table (force table fl[18][NT],
//     velocity table [VW * VH]), missing elements' reads included;
//   * every force a node sums comes from an element that exists, was computed
//     in that phase by this tile, and has the node as the expected local node,
//     in ascending element order;
//   * every LDS velocity an element phase or node phase reads was written by
//     the node phase before it; no node is written twice in one phase;
//   * the float-reciprocal node division equals integer division;
//   * over all tiles, every CG2 node is stored exactly once and every
//     element's stress exactly once, at in-range global indices;
//   * the strip order of a domain's tiles lists every tile exactly once.
// Prints "ok <cases>" and exits 0, or the first failure and exits 1.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "mevp_index.hpp"
#include "mevp_internal.hpp"

using namespace mevp;

static int g_fail = 0;
#define CHECK(cond, ...)                                   \
  do {                                                     \
    if (!(cond)) {                                         \
      if (!g_fail) {                                       \
        fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
        fprintf(stderr, __VA_ARGS__);                      \
        fprintf(stderr, "\n");                             \
      }                                                    \
      g_fail = 1;                                          \
      return;                                              \
    }                                                      \
  } while (0)

struct Domain {
  int nx, ny, NX, NY, ne, nn;
};

// One node phase: the nodes of `r`, R rounds over NT lanes, forces from the
// table of a tile whose lane (lx, ly) holds element (ex0 + lx, ey0 + ly),
// `written[slot]` telling which columns this phase computed. `seen` counts the
// nodes updated (size VW * VH for LDS output, nn for global output).
static void check_node_phase(const Domain &D, const NodeRange &r, int R, int NT, int FW,
                             int ex0, int ey0, const std::vector<char> &written,
                             std::vector<int> &seen, bool lds_out, int jx0, int jy0, int VW,
                             int VH, const std::vector<char> *vl_in) {
  const int w = r.ix1 - r.ix0, n = w * (r.iy1 - r.iy0);
  CHECK(w > 0 && r.iy1 > r.iy0, "empty node range");
  CHECK(w < 128 && R * NT <= 8192, "range %d wide, %d slots: beyond the exact float division", w,
        R * NT);
  CHECK(n <= R * NT, "%d nodes for %d lanes x %d rounds", n, NT, R);
  const float rw = 1.0f / (float)w;
  for (int tid = 0; tid < NT; ++tid)
    for (int m = 0; m < R; ++m) {
      const int k = tid + m * NT;
      const bool act = k < n;
      int dx, dy;
      node_in_range(act ? k : 0, w, rw, dx, dy);
      if (!act) {
        CHECK(dx == 0 && dy == 0, "inactive slot maps to (%d, %d)", dx, dy);
        continue;
      }
      CHECK(dx == k % w && dy == k / w, "node %d of width %d -> (%d, %d)", k, w, dx, dy);
      const int ix = r.ix0 + dx, iy = r.iy0 + dy;
      CHECK(ix >= 0 && iy >= 0 && ix < D.NX && iy < D.NY, "node (%d, %d) outside", ix, iy);
      const long j = (long)iy * D.NX + ix;
      CHECK(j >= 0 && j < D.nn, "global node %ld", j);
      const bool bnd = ix == 0 || iy == 0 || ix == D.NX - 1 || iy == D.NY - 1;
      if (lds_out) {
        const int q = (iy - jy0) * VW + (ix - jx0);
        CHECK(q >= 0 && q < VW * VH, "LDS velocity write %d of %d", q, VW * VH);
        CHECK(seen[q] == 0, "LDS node (%d, %d) written twice", ix, iy);
        seen[q]++;
      } else {
        seen[j]++;
      }
      if (vl_in && !bnd) {  // v^{p-1} from the LDS table
        const int q = (iy - jy0) * VW + (ix - jx0);
        CHECK(q >= 0 && q < VW * VH && (*vl_in)[q], "node (%d, %d) reads unwritten LDS", ix, iy);
      }
      if (bnd) continue;
      int off[4];
      bool two_x, two_y;
      node_force_offsets(ix, iy, ex0, ey0, FW, NT, off, two_x, two_y);
      const bool use[4] = {true, two_x, two_y, two_x && two_y};
      long prev = -1;
      for (int s = 0; s < 4; ++s) {
        for (int comp = 0; comp < 2; ++comp) {
          const int o = off[s] + comp * 9 * NT;
          CHECK(o >= 0 && o < 18 * NT, "force read %d outside fl[18][%d]", o, NT);
        }
        if (!use[s]) continue;
        const int row = off[s] / NT, col = off[s] % NT;
        CHECK(row < 9 && col < NT, "force read row %d col %d", row, col);
        CHECK(written[col], "node (%d, %d) sums column %d, not computed in this phase", ix, iy, col);
        const int ex = ex0 + col % FW, ey = ey0 + col / FW;
        CHECK(ex >= 0 && ey >= 0 && ex < D.nx && ey < D.ny, "element (%d, %d) outside", ex, ey);
        const int b = row / 3, c = row % 3;
        CHECK(2 * ex + c == ix && 2 * ey + b == iy,
              "node (%d, %d) reads local node %d of element (%d, %d)", ix, iy, row, ex, ey);
        const long e = (long)ey * D.nx + ex;
        CHECK(e > prev, "node (%d, %d): elements not ascending", ix, iy);
        prev = e;
      }
    }
}

template <int EX, int EY>
static void check_single(const Domain &D, std::vector<int> &node_seen, std::vector<int> &el_seen) {
  constexpr int TX = EX - 1, TY = EY - 1, NT = EX * EY;
  constexpr int R = ((2 * EX - 1) * (2 * EY - 1) + NT - 1) / NT;
  for (int y0 = 0; y0 < D.ny; y0 += TY)
    for (int x0 = 0; x0 < D.nx; x0 += TX) {
      std::vector<char> written(NT, 0);
      for (int tid = 0; tid < NT; ++tid) {
        const int lx = tid % EX, ly = tid / EX, ex = x0 - 1 + lx, ey = y0 - 1 + ly;
        if (ex >= 0 && ey >= 0 && ex < D.nx && ey < D.ny) {
          written[tid] = 1;
          if (lx > 0 && ly > 0) el_seen[(long)ey * D.nx + ex]++;
        }
      }
      const NodeRange own = owned_nodes(x0, y0, TX, TY, D.nx, D.ny, D.NX, D.NY);
      check_node_phase(D, own, R, NT, EX, x0 - 1, y0 - 1, written, node_seen, false, 0, 0, 0, 0,
                       nullptr);
      if (g_fail) return;
    }
}

template <int EX, int EY, int K>
static void check_multi(const Domain &D, std::vector<int> &node_seen, std::vector<int> &el_seen) {
  constexpr int TX = EX - 1, TY = EY - 1;
  constexpr int FX = EX + 2 * K - 2, FY = EY + 2 * K - 2, NT = FX * FY;
  constexpr int VW = 2 * TX + 4 * K - 5, VH = 2 * TY + 4 * K - 5;
  for (int y0 = 0; y0 < D.ny; y0 += TY)
    for (int x0 = 0; x0 < D.nx; x0 += TX) {
      const int ex0 = x0 - K, ey0 = y0 - K, jx0 = 2 * (ex0 + 1), jy0 = 2 * (ey0 + 1);
      std::vector<char> vl(VW * VH, 0);  // LDS velocity entries written so far
      for (int i = 0; i < K; ++i) {
        std::vector<char> written(NT, 0);
        for (int tid = 0; tid < NT; ++tid) {
          const int lx = tid % FX, ly = tid / FX, ex = ex0 + lx, ey = ey0 + ly;
          const bool exists = ex >= 0 && ey >= 0 && ex < D.nx && ey < D.ny;
          if (!(exists && lx >= i && ly >= i && lx < FX - i && ly < FY - i)) continue;
          written[tid] = 1;
          if (i > 0)  // the 3 x 3 velocity gather from the LDS table
            for (int b = 0; b < 3; ++b)
              for (int c = 0; c < 3; ++c) {
                const int q = (2 * ey - jy0) * VW + (2 * ex - jx0) + b * VW + c;
                CHECK(q >= 0 && q < VW * VH, "element (%d, %d) gathers LDS %d", ex, ey, q);
                CHECK(vl[q], "element (%d, %d) gathers a node not updated", ex, ey);
              }
          if (i == K - 1 && lx >= K && ly >= K) el_seen[(long)ey * D.nx + ex]++;
        }
        if (i < K - 1) {
          const NodeRange r = multi_phase_nodes(x0, y0, TX, TY, K, i, D.NX, D.NY);
          constexpr int R = (VW * VH + NT - 1) / NT;
          std::vector<int> seen(VW * VH, 0);
          std::vector<char> prev = vl;
          check_node_phase(D, r, R, NT, FX, ex0, ey0, written, seen, true, jx0, jy0, VW, VH,
                           i > 0 ? &prev : nullptr);
          if (g_fail) return;
          for (int q = 0; q < VW * VH; ++q) vl[q] = seen[q] > 0;
        } else {
          const NodeRange own = owned_nodes(x0, y0, TX, TY, D.nx, D.ny, D.NX, D.NY);
          constexpr int R = ((2 * EX - 1) * (2 * EY - 1) + NT - 1) / NT;
          check_node_phase(D, own, R, NT, FX, ex0, ey0, written, node_seen, false, jx0, jy0, VW,
                           VH, &vl);
          if (g_fail) return;
        }
      }
    }
}

// The strip order of a domain's tiles lists every tile of the ntx x nty grid
// exactly once, column strips of `strip` tiles left to right, rows bottom to
// top within a strip.
static void check_strip_order(int ntx, int nty, int strip) {
  std::vector<int> seen((size_t)ntx * nty, 0);
  int prev_strip = 0, prev_row = 0, prev_col = -1;
  for (int k = 0; k < ntx * nty; ++k) {
    int col, row;
    strip_tile(k, ntx, nty, strip, col, row);
    CHECK(col >= 0 && col < ntx && row >= 0 && row < nty, "tile %d of %dx%d -> (%d, %d)", k, ntx,
          nty, col, row);
    CHECK(seen[(size_t)row * ntx + col]++ == 0, "tile (%d, %d) listed twice", col, row);
    const int sj = col / strip;
    CHECK(sj > prev_strip || (sj == prev_strip && (row > prev_row ||
                                                   (row == prev_row && col > prev_col))),
          "tile %d of %dx%d out of strip order", k, ntx, nty);
    prev_strip = sj;
    prev_row = row;
    prev_col = col;
  }
}

template <int EX, int EY>
static void check_shape(const Domain &D, int K) {
  std::vector<int> node_seen(D.nn, 0), el_seen(D.ne, 0);
  if (K == 1) check_single<EX, EY>(D, node_seen, el_seen);
  if (K == 2) check_multi<EX, EY, 2>(D, node_seen, el_seen);
  if (K == 3) check_multi<EX, EY, 3>(D, node_seen, el_seen);
  if (g_fail) return;
  for (int j = 0; j < D.nn; ++j)
    CHECK(node_seen[j] == 1, "shape %dx%d K=%d: node %d stored %d times", EX, EY, K, j,
          node_seen[j]);
  for (int e = 0; e < D.ne; ++e)
    CHECK(el_seen[e] == 1, "shape %dx%d K=%d: element %d stored %d times", EX, EY, K, e,
          el_seen[e]);
}

int main() {
  static_assert(kNumTileShapes == 4, "the shapes below follow kTileShapes");
  const int sizes[][2] = {{1, 1},   {1, 37},  {37, 1},  {2, 2},   {3, 5},    {13, 13},
                          {14, 14}, {16, 14}, {17, 9},  {32, 15}, {33, 16},  {47, 31},
                          {65, 29}, {100, 3}, {128, 96}, {173, 61}};
  int cases = 0;
  for (const auto &sz : sizes) {
    Domain D;
    D.nx = sz[0];
    D.ny = sz[1];
    D.NX = 2 * D.nx + 1;
    D.NY = 2 * D.ny + 1;
    D.ne = D.nx * D.ny;
    D.nn = D.NX * D.NY;
    for (int sh = 0; sh < kNumTileShapes; ++sh) {
      const int tx = kTileShapes[sh][0] - 1, ty = kTileShapes[sh][1] - 1;
      const int strip = strip_width(tx, kStripElems);
      if (strip < 1 || strip * tx > 2 * kStripElems) {
        fprintf(stderr, "FAIL: strip of %d tiles for tiles %d wide\n", strip, tx);
        return 1;
      }
      check_strip_order((D.nx + tx - 1) / tx, (D.ny + ty - 1) / ty, strip);
    }
    for (int strip : {1, 3, 8, 16, 20}) {
      check_strip_order(65, 3, strip);
      check_strip_order(16, 5, strip);
      check_strip_order(47, 31, strip);
    }
    for (int K = 1; K <= 3; ++K) {
      check_shape<kTileShapes[0][0], kTileShapes[0][1]>(D, K);
      check_shape<kTileShapes[1][0], kTileShapes[1][1]>(D, K);
      check_shape<kTileShapes[2][0], kTileShapes[2][1]>(D, K);
      check_shape<kTileShapes[3][0], kTileShapes[3][1]>(D, K);
      if (g_fail) {
        fprintf(stderr, "domain %dx%d, %d subcycle(s) per pass\n", D.nx, D.ny, K);
        return 1;
      }
      cases += 4;
    }
  }
  printf("ok %d\n", cases);
  return 0;
}
