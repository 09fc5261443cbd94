// tile2_geometry_check.hip -- host-side check of the two-step tile geometry
// (TileGeom2 in heat_tile2.hpp, host-callable), run by
// tests/test_tile2_geometry.py before any kernel runs.  For every thread of
// every tile of ragged and row-padded shapes it checks that
//   * every global offset is in bounds and aligned to a lane;
//   * every LDS slot read by an updated node's stencil (both steps) holds
//     exactly the neighbour it needs, and an intermediate value read there
//     was updated exactly when that neighbour is interior;
//   * no LDS slot is written with two different nodes;
//   * every interior node is stored exactly once, and masked stores only
//     touch non-interior nodes.
// Prints the problems it finds and exits non-zero if there are any.
#include "heat_tile2.hpp"
#include <cstdio>
#include <map>
#include <set>
#include <vector>
using namespace hc;

struct Tag { int i, j; bool set; int writer; bool upd; };

template <int VEC, int TXL, int BY>
int check(int nx, int ny, int nz, int pitch = 0) {
    if (pitch == 0) pitch = nx;
    using G = TileGeom2<VEC, TXL, BY>;
    const int TX = G::TX;
    const int ntx = (nx + TX - 1) / TX, nty = (ny - 2 + BY - 1) / BY;
    const long long plane = (long long)pitch * ny;
    int bad = 0;
    std::vector<int> stored((size_t)plane, 0);
    auto coord = [&](long long off, int v) { long long o = off + v; return std::make_pair((int)(o % pitch), (int)(o / pitch)); };
    auto interior = [&](int i, int j) { return i >= 1 && i <= nx - 2 && j >= 1 && j <= ny - 2; };
    for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) {
            std::vector<G> gs;
            for (int t = 0; t < G::NT; ++t) gs.emplace_back(t, nx, pitch, ny, nz, tx, ty, 1, nz - 2);
            std::vector<Tag> U(G::U_ELEMS, Tag{0, 0, false, -1, false}), A(G::A_ELEMS, Tag{0, 0, false, -1, false});
            auto wr = [&](std::vector<Tag> &L, int slot, int i, int j, int t, const char *what, bool upd = false) {
                if (slot < 0 || slot >= (int)L.size()) { printf("LDS write OOB %s slot %d t %d\n", what, slot, t); ++bad; return; }
                if (&L == &A && slot == G::A_ELEMS - 1) return;  // sink
                if (L[slot].set && L[slot].writer != t && (L[slot].i != i || L[slot].j != j)) {
                    printf("LDS conflict %s slot %d: (%d,%d) by %d vs (%d,%d) by %d\n", what, slot, L[slot].i, L[slot].j, L[slot].writer, i, j, t); ++bad; }
                L[slot] = Tag{i, j, true, t, upd};
            };
            auto chk_off = [&](long long off, const char *what, int t) {
                if (off < 0 || off + VEC > plane || off % VEC) { printf("global OOB/misaligned %s off %lld t %d tile %d,%d\n", what, off, t, tx, ty); ++bad; }
            };
            // writes of the u^t plane
            for (int t = 0; t < G::NT; ++t) {
                const G &g = gs[t];
                chk_off(g.own, "own", t); chk_off(g.r1, "r1", t); chk_off(g.r2, "r2", t);
                for (int v = 0; v < VEC; ++v) { auto c = coord(g.own, v); wr(U, g.own_u + v * TXL, c.first, c.second, t, "U own"); }
                if (g.r1on) {
                    if (g.r1vec) for (int v = 0; v < VEC; ++v) { auto c = coord(g.r1, v); wr(U, g.r1_u + v * TXL, c.first, c.second, t, "U r1"); }
                    else { auto c = coord(g.r1, g.r1sel); wr(U, g.r1_u, c.first, c.second, t, "U r1c"); }
                }
                if (g.r2on) {
                    if (g.r2vec) for (int v = 0; v < VEC; ++v) { auto c = coord(g.r2, v); wr(U, g.r2_u + v * TXL, c.first, c.second, t, "U r2"); }
                    else { auto c = coord(g.r2, g.r2sel); wr(U, g.r2_u, c.first, c.second, t, "U r2c"); }
                }
            }
            auto need = [&](std::vector<Tag> &L, int slot, int i, int j, const char *what, int t) {
                if (slot < 0 || slot >= (int)L.size()) { printf("LDS read OOB %s slot %d t %d\n", what, slot, t); ++bad; return; }
                if (!L[slot].set || L[slot].i != i || L[slot].j != j || (&L == &A && L[slot].upd != interior(i, j))) {
                    printf("tile %d,%d t %d %s slot %d holds (%d,%d)%s, needs (%d,%d)\n", tx, ty, t, what, slot, L[slot].i, L[slot].j, L[slot].set ? "" : " unset", i, j); ++bad; }
            };
            auto rd_ok = [&](std::vector<Tag> &L, int slot, const char *what, int t) {
                if (slot < 0 || slot >= (int)L.size()) { printf("LDS read OOB %s slot %d t %d\n", what, slot, t); ++bad; }
            };
            // step A at the own nodes and the inner-ring elements; writes of the A plane
            for (int t = 0; t < G::NT; ++t) {
                const G &g = gs[t];
                for (int v = 0; v < VEC; ++v) {
                    rd_ok(U, g.own_u + v * TXL - G::LDU, "A y-", t); rd_ok(U, g.own_u + v * TXL + G::LDU, "A y+", t);
                    rd_ok(U, g.r1_u + v * TXL - G::LDU, "A1 y-", t); rd_ok(U, g.r1_u + v * TXL + G::LDU, "A1 y+", t);
                }
                rd_ok(U, g.xm_u, "xm", t); rd_ok(U, g.xp_u, "xp", t); rd_ok(U, g.r1xm_u, "r1xm", t); rd_ok(U, g.r1xp_u, "r1xp", t);
                for (int v = 0; v < VEC; ++v) {
                    auto c = coord(g.own, v);
                    const bool upd = g.st[v];
                    if (upd != interior(c.first, c.second) && upd) { printf("core mask set on non-interior (%d,%d)\n", c.first, c.second); ++bad; }
                    if (upd) {
                        if (v == 0) need(U, g.xm_u, c.first - 1, c.second, "A core xm", t);
                        if (v == VEC - 1) need(U, g.xp_u, c.first + 1, c.second, "A core xp", t);
                        need(U, g.own_u + v * TXL - G::LDU, c.first, c.second - 1, "A core y-", t);
                        need(U, g.own_u + v * TXL + G::LDU, c.first, c.second + 1, "A core y+", t);
                    }
                    wr(A, g.own_a + v * TXL, c.first, c.second, t, "A own", g.st[v]);
                }
                // a core node that is interior must be updated, unless it is a redirected lane
                for (int v = 0; v < VEC; ++v) {
                    auto c = coord(g.own, v);
                    const int i = tx * TX + (t % TXL) * VEC + v, j = 1 + ty * BY + t / TXL;
                    if (interior(i, j) && !g.st[v]) { printf("interior (%d,%d) not updated\n", i, j); ++bad; }
                    if (g.st[v] && (c.first != i || c.second != j)) { printf("updated node at wrong address\n"); ++bad; }
                    if (g.st[v]) stored[(size_t)j * pitch + i]++;
                    else if (interior(c.first, c.second)) { printf("masked store to interior (%d,%d)\n", c.first, c.second); ++bad; }
                }
                if (g.r1on) {
                    const int nn = g.r1vec ? VEC : 1;
                    for (int v = 0; v < nn; ++v) {
                        auto c = g.r1vec ? coord(g.r1, v) : coord(g.r1, g.r1sel);
                        // the intended coordinate of this ring element
                        const bool upd = g.r1st[v];
                        if (upd && !interior(c.first, c.second)) { printf("ring mask on non-interior\n"); ++bad; }
                        if (upd) {
                            if (v == 0) need(U, g.r1xm_u, c.first - 1, c.second, "A ring xm", t);
                            if (v == nn - 1 || !g.r1vec) need(U, g.r1xp_u, c.first + 1, c.second, "A ring xp", t);
                            need(U, g.r1_u + v * TXL - G::LDU, c.first, c.second - 1, "A ring y-", t);
                            need(U, g.r1_u + v * TXL + G::LDU, c.first, c.second + 1, "A ring y+", t);
                        }
                        wr(A, g.r1_a + v * TXL, c.first, c.second, t, "A ring", g.r1st[v]);
                    }
                }
            }
            // step B at the own nodes
            for (int t = 0; t < G::NT; ++t) {
                const G &g = gs[t];
                for (int v = 0; v < VEC; ++v) {
                    rd_ok(A, g.own_a + v * TXL - G::LDA, "B y-", t); rd_ok(A, g.own_a + v * TXL + G::LDA, "B y+", t);
                    if (!g.st[v]) continue;
                    auto c = coord(g.own, v);
                    if (v == 0) need(A, g.xm_a, c.first - 1, c.second, "B xm", t);
                    if (v == VEC - 1) need(A, g.xp_a, c.first + 1, c.second, "B xp", t);
                    need(A, g.own_a + v * TXL - G::LDA, c.first, c.second - 1, "B y-", t);
                    need(A, g.own_a + v * TXL + G::LDA, c.first, c.second + 1, "B y+", t);
                }
            }
        }
    for (int j = 1; j <= ny - 2; ++j)
        for (int i = 1; i <= nx - 2; ++i)
            if (stored[(size_t)j * pitch + i] != 1) { if (bad < 50) printf("node (%d,%d) stored %d times\n", i, j, stored[(size_t)j * pitch + i]); ++bad; }
    return bad;
}

// The z-plan of a run: every output plane of [kb, ke] is written, nothing
// outside the interior planes [1, nz-2] is, and the march reads planes
// within two of what it writes (plus its prefetch, clamped).
static int check_run_plans() {
    int bad = 0;
    for (int nz = 3; nz <= 140; ++nz)
        for (int zb : {16, 32, 64})
            for (int kb = 1; kb <= nz - 2; ++kb)
                for (int ke = kb; ke <= nz - 2; ++ke) {
                    const hc::RunPlan p = hc::run_plan(kb, ke, zb);
                    std::vector<int> w(nz, 0);
                    for (int k = p.start; k < p.start + p.m * zb; ++k) {
                        if (k < 0 || k >= nz) { ++bad; continue; }
                        ++w[k];
                    }
                    for (int k = p.rest; k <= ke; ++k) ++w[k];
                    for (int k = 0; k < nz; ++k) {
                        const bool in_run = k >= kb && k <= ke;
                        if (in_run && w[k] != 1) ++bad;
                        if (w[k] && (k < 1 || k > nz - 2)) ++bad;
                        if (!in_run && w[k] && k > ke) ++bad;  // never past the run
                    }
                    if (p.m > 0 && p.start > kb) ++bad;
                    if (bad && bad < 5)
                        printf("run plan nz %d zb %d [%d, %d]: start %d m %d rest %d\n", nz, zb,
                               kb, ke, p.start, p.m, p.rest);
                }
    printf("run plans: %d problems\n", bad);
    return bad;
}

int main() {
    int bad = check_run_plans();
    const int dims[][2] = {{3, 3}, {5, 4}, {130, 9}, {67, 33}, {264, 19}, {512, 512}, {1029, 6}, {64, 131}, {258, 40}, {520, 70}};
    for (auto &d : dims) {
        const int nx = d[0], ny = d[1], nz = 7;
        int b = 0;
        b += check<1, 256, 4>(nx, ny, nz); b += check<1, 64, 4>(nx, ny, nz);
        if (nx % 2 == 0) { b += check<2, 64, 8>(nx, ny, nz); b += check<2, 64, 16>(nx, ny, nz); b += check<2, 128, 4>(nx, ny, nz);
                           b += check<2, 128, 8>(nx, ny, nz); b += check<2, 256, 4>(nx, ny, nz); }
        if (nx % 4 == 0) { b += check<4, 64, 8>(nx, ny, nz); b += check<4, 64, 16>(nx, ny, nz); b += check<4, 128, 4>(nx, ny, nz); b += check<4, 128, 8>(nx, ny, nz); }
        if (nx % 8 == 0) { b += check<8, 64, 8>(nx, ny, nz); b += check<8, 64, 4>(nx, ny, nz); }
        printf("%d x %d: %d problems\n", nx, ny, b);
        bad += b;
    }
    // batch width classes (rows padded to 16 bytes)
    const int bd[][2] = {{32, 32}, {33, 40}, {61, 35}, {100, 99}, {129, 50}, {192, 192}, {37, 191}, {150, 33},
                         {28, 21}, {40, 9}, {64, 13}, {130, 17}, {97, 66}, {96, 30},
                         {31, 20}, {103, 12}, {67, 9}};
    for (auto &d : bd) {
        const int nx = d[0], ny = d[1], nz = 6;
        int b = 0;
        const int p4 = (nx + 3) / 4 * 4, p2 = (nx + 1) / 2 * 2, p8 = (nx + 7) / 8 * 8;
        b += check<4, 8, 64>(nx, ny, nz, p4); b += check<4, 16, 32>(nx, ny, nz, p4); b += check<4, 32, 16>(nx, ny, nz, p4);
        b += check<4, 64, 8>(nx, ny, nz, p4); b += check<4, 128, 4>(nx, ny, nz, p4); b += check<4, 8, 32>(nx, ny, nz, p4);
        b += check<4, 16, 16>(nx, ny, nz, p4); b += check<4, 32, 8>(nx, ny, nz, p4); b += check<4, 64, 4>(nx, ny, nz, p4);
        b += check<4, 16, 64>(nx, ny, nz, p4); b += check<4, 128, 8>(nx, ny, nz, p4);
        b += check<2, 8, 64>(nx, ny, nz, p2); b += check<2, 128, 4>(nx, ny, nz, p2);
        b += check<8, 8, 64>(nx, ny, nz, p8); b += check<8, 128, 4>(nx, ny, nz, p8);
        printf("batch %d x %d: %d problems\n", nx, ny, b);
        bad += b;
    }
    printf(bad ? "FAIL\n" : "ALL OK\n");
    return bad ? 1 : 0;
}
