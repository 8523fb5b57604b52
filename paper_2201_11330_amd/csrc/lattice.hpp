// Discrete velocity sets for the device code, generated at compile time.
//
// Sec. 2.1 numbers D2Q9 lexicographically in (e_x, e_y) with e_x slowest,
// which makes the opposite of direction a equal to Q - 1 - a.  The same rule
// in three dimensions (e_x slowest, then e_y, then e_z), restricted to the
// 19 velocities of Qian's D3Q19 (|e|^2 <= 2), keeps that property.  Weights
// follow |e|^2: D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36.
#pragma once

namespace imexlbm {

template <int DIM>
struct Lattice {
    static constexpr int D = DIM;
    static constexpr int Q = DIM == 2 ? 9 : 19;
    int e[Q][3];
    double w[Q];

    static constexpr double weight(int norm2)
    {
        if (DIM == 2) return norm2 == 0 ? 4.0 / 9.0 : (norm2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        return norm2 == 0 ? 1.0 / 3.0 : (norm2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }

    static constexpr Lattice make()
    {
        Lattice L{};
        int a = 0;
        const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
        for (int ex = -1; ex <= 1; ++ex)
            for (int ey = -1; ey <= 1; ++ey)
                for (int ez = zlo; ez <= zhi; ++ez) {
                    const int n2 = ex * ex + ey * ey + ez * ez;
                    if (n2 > 2) continue;
                    L.e[a][0] = ex;
                    L.e[a][1] = ey;
                    L.e[a][2] = ez;
                    L.w[a] = weight(n2);
                    ++a;
                }
        return L;
    }

    static constexpr int opp(int a) { return Q - 1 - a; }
};

template <int DIM>
inline constexpr Lattice<DIM> kLattice = Lattice<DIM>::make();

// Compile-time checks of the generated sets: count, opposite index, weights
// summing to one and the second moment c_s^2 = 1/3.
template <int DIM>
constexpr bool lattice_ok()
{
    constexpr auto L = kLattice<DIM>;
    double sw = 0.0, sxx = 0.0;
    for (int a = 0; a < L.Q; ++a) {
        for (int d = 0; d < 3; ++d)
            if (L.e[L.opp(a)][d] != -L.e[a][d]) return false;
        sw += L.w[a];
        sxx += L.w[a] * L.e[a][0] * L.e[a][0];
    }
    const double eps = 1e-15;
    return (sw - 1.0 < eps && 1.0 - sw < eps) && (sxx - 1.0 / 3 < eps && 1.0 / 3 - sxx < eps);
}
static_assert(lattice_ok<2>(), "D2Q9 table");
static_assert(lattice_ok<3>(), "D3Q19 table");
static_assert(kLattice<2>.e[0][0] == -1 && kLattice<2>.e[0][1] == -1 && kLattice<2>.e[4][0] == 0,
              "D2Q9 numbering of Sec. 2.1");
static_assert(kLattice<3>.e[9][0] == 0 && kLattice<3>.e[9][1] == 0 && kLattice<3>.e[9][2] == 0,
              "D3Q19 rest direction in the middle");

}  // namespace imexlbm
