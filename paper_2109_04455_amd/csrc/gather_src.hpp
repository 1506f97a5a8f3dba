// Source offsets of the D2Q5 gathers (forward ADR step and its adjoint),
// shared by the kernels and by a host-compiled bounds check: this header
// depends on nothing but the compiler, so the same functions build for the
// GPU and for the host.
//
// A species' five post-collision planes form one block: plane d starts
// d * PB bytes after the block base, rows are RB bytes apart, B is the size
// of one population and node (x, y) sits at byte offset o = (y * nxp + x) * B
// within a plane.  Mask bits 0..3 mark a solid neighbour east, north, west,
// south (rows outside the lattice count as solid, columns outside it as the
// open inlet and outlet).  Paper: Sec. "Lattice-Boltzmann for
// Advection-Diffusion-Reaction" (pull streaming), Sec. "Boundary conditions
// and flux computation in ADE", Eq. BC (bounce-back, inlet and outlet rules).
#pragma once

#if defined(__HIPCC__)
#define LBF_HD __host__ __device__
#else
#define LBF_HD
#endif

namespace lbf {
namespace gather {

constexpr unsigned BIT_E = 1u, BIT_N = 2u, BIT_W = 4u, BIT_S = 8u;
enum { DE = 1, DN = 2, DW = 3, DS = 4 };

// Forward step: population i of node x arrives from x - c_i, or is the
// node's own opposite population when x - c_i is solid (bounce-back) or x is
// the inlet (E, anti-bounce-back on the node's own W); at the outlet W is
// rebuilt from the node's own populations, so its slot reads the node's own
// E (the rule's last term; the other own populations are read apart).
template <typename Off>
LBF_HD inline void adr_sources(Off B, Off PB, Off RB, Off o, int x, int nx, unsigned m,
                               Off (&src)[5])
{
    const Off oE = o + DE * PB, oN = o + DN * PB, oW = o + DW * PB, oS = o + DS * PB;
    const bool in = x == 0, out = x == nx - 1;
    src[0] = o;
    src[DE] = (in || (m & BIT_W)) ? oW : oE - B;
    src[DN] = (m & BIT_S) ? oS : oN - RB;
    src[DW] = (out || (m & BIT_E)) ? oE : oW + B;
    src[DS] = (m & BIT_N) ? oN : oS + RB;
}

// Adjoint step (the transpose of the streaming above): the post-collision
// population i of node x fed g_i(x + c_i), or g_opp(i)(x) by bounce-back, or
// at the inlet (W) g_E(x) and at the outlet (E) the node's own g_W.
template <typename Off>
LBF_HD inline void adj_sources(Off B, Off PB, Off RB, Off o, int x, int nx, unsigned m,
                               Off (&src)[5])
{
    const Off oE = o + DE * PB, oN = o + DN * PB, oW = o + DW * PB, oS = o + DS * PB;
    const bool in = x == 0, out = x == nx - 1;
    src[0] = o;
    src[DE] = (out || (m & BIT_E)) ? oW : oE + B;
    src[DN] = (m & BIT_N) ? oS : oN + RB;
    src[DW] = (in || (m & BIT_W)) ? oE : oW - B;
    src[DS] = (m & BIT_S) ? oN : oS - RB;
}

}  // namespace gather
}  // namespace lbf
