// Host build of the library's lattice index helpers (wd_device.hpp), for tests/test_index_map.py.
// Prints, for one lattice, every (parity, checkerboard index) with its lexicographic site and the
// checkerboard indices of its 8 neighbours (nb_index, checked equal to nb_from_cb), then the FP16 site scale rule on chosen magnitudes.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>

#include "wd_device.hpp"

using namespace wd;

// both neighbour-index forms of the library: they must agree (the probe exits with status 3 if not)
template <int MU, int D>
static int nb(const Geo& g, int cb, int x, int y, int z, int t)
{
    const int a = nb_index<MU, D>(g, x, y, z, t), b = nb_from_cb<MU, D>(g, cb, x, y, z, t);
    if (a != b) {
        std::fprintf(stderr, "nb_index %d != nb_from_cb %d (mu %d, d %d, cb %d)\n", a, b, MU, D, cb);
        std::exit(3);
    }
    return a;
}

int main(int argc, char** argv)
{
    if (argc != 5) return 2;
    Geo g{};
    g.X = std::atoi(argv[1]);
    g.Y = std::atoi(argv[2]);
    g.Z = std::atoi(argv[3]);
    g.T = std::atoi(argv[4]);
    g.Xh = g.X / 2;
    g.Vh = g.X * g.Y * g.Z * g.T / 2;
    for (int p = 0; p < 2; p++)
        for (int cb = 0; cb < g.Vh; cb++) {
            int x, y, z, t;
            cb_coords(g, p, cb, x, y, z, t);
            const long n = x + (long)g.X * (y + (long)g.Y * (z + (long)g.Z * t));
            std::printf("S %d %d %ld %d %d %d %d %d %d %d %d %d\n", p, cb, n, cb_index(g, x, y, z, t),
                        nb<0, 0>(g, cb, x, y, z, t), nb<0, 1>(g, cb, x, y, z, t), nb<1, 0>(g, cb, x, y, z, t),
                        nb<1, 1>(g, cb, x, y, z, t), nb<2, 0>(g, cb, x, y, z, t), nb<2, 1>(g, cb, x, y, z, t),
                        nb<3, 0>(g, cb, x, y, z, t), nb<3, 1>(g, cb, x, y, z, t));
        }
    const float ms[] = {0.0f, 1e-45f, 1e-39f, std::numeric_limits<float>::min(), 1e-20f, 1.0f, 3e38f,
                        std::numeric_limits<float>::infinity(), std::numeric_limits<float>::quiet_NaN()};
    for (float m : ms) std::printf("F %.9g %.9g\n", (double)m, (double)f16_site_inv(m));
    return 0;
}
