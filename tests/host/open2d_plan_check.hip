// Host-side check of the one-launch 2D open step's work split (no GPU code runs): for every box
// from 3 x 3 to 45 x 45 cells, the network segments own every ring cell exactly once, each
// segment's rows fit one 16-row tile and name valid face nodes, and every face node a ring cell
// pulls a prediction from (D2Q9 velocities, which include those of D2Q5) sits at the row the
// kernel looks up.  Exit status 0 when every check holds.
#include <cstdio>
#include <vector>

#include "open_bc.hpp"

using namespace lbm;

int main() {
    long long checks = 0, bad = 0;
    const int C[9][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1}, {1, -1}, {-1, 1}, {1, 1}};
    for (int nx = 3; nx <= 45; ++nx)
        for (int ny = 3; ny <= 45; ++ny) {
            std::vector<int> own(nx * ny, 0), ring(nx * ny, 0);
            const int n[3] = {nx, ny, 1};
            for (int w = 0; w < open2d_segments(nx, ny); ++w) {
                const OpenSeg sg = open2d_segment(w, nx, ny);
                const OpenRows r = open2d_rows(sg, nx, ny);
                ++checks;
                if (r.nrows > 16 || sg.m < 1 || sg.m > kOpenSeg) ++bad;
                for (int j = 0; j < r.nrows; ++j) {
                    int f, p;
                    open2d_row_node(r, j, nx, f, p);
                    ++checks;
                    if (f < 0 || f > 3 || p < 0 || p >= (f < 2 ? ny : nx)) ++bad;
                }
                for (int l = 0; l < sg.m; ++l) {
                    int x[3] = {0, 0, 0};
                    const int a = sg.f >> 1;
                    x[a] = (sg.f & 1) ? n[a] - 1 : 0;
                    x[1 - a] = sg.p0 + l;
                    own[x[1] * nx + x[0]]++;
                    for (int i = 1; i < 9; ++i) {
                        const int sp[3] = {x[0] - C[i][0], x[1] - C[i][1], 0};
                        int cl[3];
                        for (int b = 0; b < 3; ++b) cl[b] = sp[b] < 0 ? 0 : (sp[b] > n[b] - 1 ? n[b] - 1 : sp[b]);
                        for (int b = 0; b < 2; ++b) {
                            if (sp[b] == cl[b]) continue;
                            const int fb = 2 * b + (sp[b] > cl[b] ? 1 : 0);
                            const int row = open2d_row_of(r, fb, cl, nx);
                            ++checks;
                            if (row < 0 || row >= r.nrows) {
                                ++bad;
                                continue;
                            }
                            int f, p;
                            open2d_row_node(r, row, nx, f, p);
                            if (f != fb || p != (fb < 2 ? cl[1] : cl[0])) ++bad;
                        }
                    }
                }
            }
            for (long long c = 0; c < 2LL * ny + 2LL * (nx - 2); ++c) {
                int x[3];
                open2d_ring_cell(c, nx, ny, x);
                ring[x[1] * nx + x[0]]++;
            }
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const int want = (x == 0 || x == nx - 1 || y == 0 || y == ny - 1) ? 1 : 0;
                    ++checks;
                    if (own[y * nx + x] != want || ring[y * nx + x] != want) ++bad;
                }
        }
    std::printf("checks %lld bad %lld\n", checks, bad);
    return bad != 0;
}
