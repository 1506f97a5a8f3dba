// Host build of the D2Q5 gather source offsets (paper_2109_04455_amd/csrc/
// gather_src.hpp, the functions the kernels call): every offset of every
// node of small lattices, for every bounce-back mask the mask builder can
// give it, must lie inside its species' block of five planes and be aligned
// to one population.  Prints "ok" and returns 0, else the first failures.
#include <cstdint>
#include <cstdio>
#include <initializer_list>

#include "gather_src.hpp"

using namespace lbf::gather;

template <typename Off>
long check(int nx, int ny, int nxp, Off B, long &cases)
{
    const Off RB = (Off)nxp * B, PB = (Off)ny * RB, block = 5 * PB;
    long bad = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (unsigned m = 0; m < 16; ++m) {
                // rows outside the lattice are solid neighbours
                if (y == 0 && !(m & BIT_S)) continue;
                if (y == ny - 1 && !(m & BIT_N)) continue;
                const Off o = ((Off)y * nxp + x) * B;
                Off f[5], a[5];
                adr_sources<Off>(B, PB, RB, o, x, nx, m, f);
                adj_sources<Off>(B, PB, RB, o, x, nx, m, a);
                for (int i = 0; i < 5; ++i)
                    for (const Off v : {f[i], a[i]})
                        if (v > block - B || v % B != 0) {
                            if (bad < 5)
                                std::printf("out of block: nx %d ny %d x %d y %d mask %u i %d "
                                            "offset %llu block %llu\n",
                                            nx, ny, x, y, m, i, (unsigned long long)v,
                                            (unsigned long long)block);
                            ++bad;
                        }
                ++cases;
            }
    return bad;
}

int main()
{
    const int shapes[][3] = {{8, 3, 64}, {64, 5, 64}, {70, 9, 128}, {130, 4, 192}};
    long bad = 0, cases = 0;
    for (const auto &s : shapes) {
        bad += check<uint32_t>(s[0], s[1], s[2], 4u, cases);
        bad += check<uint64_t>(s[0], s[1], s[2], 4u, cases);
        bad += check<uint64_t>(s[0], s[1], s[2], 8u, cases);
    }
    if (bad) {
        std::printf("%ld of %ld cases out of bounds\n", bad, cases);
        return 1;
    }
    std::printf("ok %ld cases\n", cases);
    return 0;
}
