// tile_geometry_check.hip -- host-side check of the single-step tile
// geometry (TileGeom in heat_tile.hpp, host-callable), run by
// tests/test_tile2_geometry.py before any kernel runs.  For every thread of
// every tile of ragged and row-padded shapes (the single-problem shapes and
// every batch width class) it checks that
//   * every global offset is in bounds and aligned to a lane;
//   * every neighbour an updated node reads -- from the LDS tile or from
//     its own lane's registers -- is exactly that neighbour;
//   * no LDS slot is written with two different nodes;
//   * every interior node is stored exactly once, and masked stores only
//     touch non-interior nodes.
// Prints the problems it finds and exits non-zero if there are any.
#include "heat_tile.hpp"
#include <cstdio>
#include <vector>
using namespace hc;

struct Tag { int i, j; bool set; int writer; };

template <int VEC, int TXL, int BY>
int check(int nx, int ny, int pitch = 0) {
    if (pitch == 0) pitch = nx;
    using G = TileGeom<VEC, TXL, BY>;
    const int TX = G::TX, LD = G::LD;
    const int ntx = (nx + TX - 1) / TX, nty = (ny - 2 + BY - 1) / BY;
    const long long plane = (long long)pitch * ny;
    const int slots = (BY + 2) * LD;
    int bad = 0;
    std::vector<int> stored((size_t)plane, 0);
    auto coord = [&](long long off, int v) { long long o = off + v; return std::make_pair((int)(o % pitch), (int)(o / pitch)); };
    auto interior = [&](int i, int j) { return i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2; };
    for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) {
            std::vector<G> gs;
            for (int t = 0; t < G::NT; ++t) gs.emplace_back(t, nx, pitch, ny, tx, ty, 1, 1);
            std::vector<Tag> L(slots, Tag{0, 0, false, -1});
            auto wr = [&](int slot, int i, int j, int t, const char *what) {
                if (slot < 0 || slot >= slots) { printf("LDS write OOB %s slot %d t %d\n", what, slot, t); ++bad; return; }
                if (L[slot].set && L[slot].writer != t && (L[slot].i != i || L[slot].j != j)) {
                    printf("LDS conflict %s slot %d: (%d,%d) vs (%d,%d)\n", what, slot, L[slot].i, L[slot].j, i, j); ++bad; }
                L[slot] = Tag{i, j, true, t};
            };
            auto chk_off = [&](long long off, const char *what, int t) {
                if (off < 0 || off + VEC > plane || off % VEC) { printf("global OOB/misaligned %s off %lld t %d tile %d,%d\n", what, off, t, tx, ty); ++bad; }
            };
            for (int t = 0; t < G::NT; ++t) {
                const G &g = gs[t];
                chk_off(g.own, "own", t); chk_off(g.ring, "ring", t);
                for (int v = 0; v < VEC; ++v) { auto c = coord(g.own, v); wr(g.own_slot + v * TXL, c.first, c.second, t, "own"); }
                if (g.rslot >= 0) {
                    if (g.rvec) for (int v = 0; v < VEC; ++v) { auto c = coord(g.ring, v); wr(g.rslot + v * TXL, c.first, c.second, t, "ring"); }
                    else { auto c = coord(g.ring, g.rsel); wr(g.rslot, c.first, c.second, t, "ring col"); }
                }
            }
            auto need = [&](int slot, int i, int j, const char *what, int t) {
                if (slot < 0 || slot >= slots) { printf("LDS read OOB %s slot %d t %d\n", what, slot, t); ++bad; return; }
                if (!L[slot].set || L[slot].i != i || L[slot].j != j) {
                    printf("tile %d,%d t %d %s slot %d holds (%d,%d)%s, needs (%d,%d)\n", tx, ty, t, what, slot, L[slot].i, L[slot].j, L[slot].set ? "" : " unset", i, j); ++bad; }
            };
            for (int t = 0; t < G::NT; ++t) {
                const G &g = gs[t];
                for (int v = 0; v < VEC; ++v) {
                    const int sl = g.own_slot + v * TXL;
                    if (sl - LD < 0 || sl + LD >= slots) { printf("LDS read OOB y t %d\n", t); ++bad; }
                    auto c = coord(g.own, v);
                    const int i = tx * TX + (t % TXL) * VEC + v, j = 1 + ty * BY + t / TXL;
                    if (interior(i, j) && !g.st[v]) { printf("interior (%d,%d) not updated\n", i, j); ++bad; }
                    if (!g.st[v]) {
                        if (interior(c.first, c.second)) { printf("masked store to interior (%d,%d)\n", c.first, c.second); ++bad; }
                        continue;
                    }
                    if (c.first != i || c.second != j) { printf("updated node at wrong address\n"); ++bad; }
                    stored[(size_t)j * pitch + i]++;
                    if (v == 0) need(g.xm_slot, i - 1, j, "xm", t);
                    else if (coord(g.own, v - 1) != std::make_pair(i - 1, j)) { printf("x- register is not (%d,%d)\n", i - 1, j); ++bad; }
                    if (v == VEC - 1) need(g.xp_slot, i + 1, j, "xp", t);
                    else if (coord(g.own, v + 1) != std::make_pair(i + 1, j)) { printf("x+ register is not (%d,%d)\n", i + 1, j); ++bad; }
                    need(sl - LD, i, j - 1, "y-", t);
                    need(sl + LD, i, j + 1, "y+", t);
                }
            }
        }
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i)
            if (stored[(size_t)j * pitch + i] != 1) { if (bad < 50) printf("node (%d,%d) stored %d times\n", i, j, stored[(size_t)j * pitch + i]); ++bad; }
    return bad;
}

int main() {
    int bad = 0;
    const int dims[][2] = {{3, 3}, {5, 4}, {130, 9}, {67, 33}, {264, 19}, {512, 512}, {1029, 6}, {64, 131}};
    for (auto &d : dims) {
        const int nx = d[0], ny = d[1];
        int b = 0;
        b += check<1, 256, 4>(nx, ny); b += check<1, 64, 4>(nx, ny);
        if (nx % 2 == 0) { b += check<2, 64, 8>(nx, ny); b += check<2, 128, 4>(nx, ny); b += check<2, 256, 4>(nx, ny); }
        if (nx % 4 == 0) { b += check<4, 64, 8>(nx, ny); b += check<4, 128, 4>(nx, ny); }
        if (nx % 8 == 0) { b += check<8, 64, 4>(nx, ny); }
        printf("%d x %d: %d problems\n", nx, ny, b);
        bad += b;
    }
    // batch width classes: rows padded to 16 bytes
    const int bd[][2] = {{32, 32}, {33, 40}, {61, 35}, {100, 99}, {129, 50}, {192, 192}, {37, 191},
                         {150, 33}, {28, 21}, {40, 9}, {64, 13}, {130, 17}, {97, 66}, {96, 30},
                         {31, 20}, {103, 12}, {67, 9}};
    for (auto &d : bd) {
        const int nx = d[0], ny = d[1];
        int b = 0;
        const int p2 = (nx + 1) / 2 * 2, p4 = (nx + 3) / 4 * 4, p8 = (nx + 7) / 8 * 8;
        b += check<4, 8, 64>(nx, ny, p4); b += check<4, 16, 32>(nx, ny, p4); b += check<4, 32, 16>(nx, ny, p4);
        b += check<4, 64, 8>(nx, ny, p4); b += check<4, 128, 4>(nx, ny, p4); b += check<4, 8, 32>(nx, ny, p4);
        b += check<4, 16, 16>(nx, ny, p4); b += check<4, 32, 8>(nx, ny, p4); b += check<4, 64, 4>(nx, ny, p4);
        b += check<4, 16, 64>(nx, ny, p4); b += check<4, 128, 8>(nx, ny, p4);
        b += check<2, 8, 64>(nx, ny, p2); b += check<2, 128, 4>(nx, ny, p2);
        b += check<8, 8, 64>(nx, ny, p8); b += check<8, 128, 4>(nx, ny, p8);
        printf("batch %d x %d: %d problems\n", nx, ny, b);
        bad += b;
    }
    printf(bad ? "FAIL\n" : "ALL OK\n");
    return bad ? 1 : 0;
}
