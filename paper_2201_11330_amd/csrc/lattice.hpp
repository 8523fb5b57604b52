// Discrete velocity sets for the device code, generated at compile time.
//
// Sec. 2.1 numbers D2Q9 lexicographically in (e_x, e_y) with e_x slowest,
// which makes the opposite of direction a equal to Q - 1 - a.  The same rule
// in three dimensions (e_x slowest, then e_y, then e_z) gives D3Q27 over all
// of {-1,0,1}^3 and, restricted to |e|^2 <= 2, Qian's D3Q19; both keep the
// opposite-index property.  Weights follow |e|^2: D2Q9 4/9, 1/9, 1/36;
// D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216.
//
// The template argument is the lattice kind of the C interface:
// 0 = D2Q9, 1 = D3Q19, 2 = D3Q27.
#pragma once

namespace imexlbm {

template <int KIND>
struct Lattice {
    static constexpr int D = KIND == 0 ? 2 : 3;
    static constexpr int Q = KIND == 0 ? 9 : (KIND == 1 ? 19 : 27);
    static constexpr int kMaxNorm2 = KIND == 2 ? 3 : 2;
    int e[Q][3];
    double w[Q];

    static constexpr double weight(int norm2)
    {
        if (KIND == 0) return norm2 == 0 ? 4.0 / 9.0 : (norm2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        if (KIND == 1) return norm2 == 0 ? 1.0 / 3.0 : (norm2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        return norm2 == 0 ? 8.0 / 27.0
                          : (norm2 == 1 ? 2.0 / 27.0 : (norm2 == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
    }

    static constexpr Lattice make()
    {
        Lattice L{};
        int a = 0;
        const int zlo = D == 3 ? -1 : 0, zhi = D == 3 ? 1 : 0;
        for (int ex = -1; ex <= 1; ++ex)
            for (int ey = -1; ey <= 1; ++ey)
                for (int ez = zlo; ez <= zhi; ++ez) {
                    const int n2 = ex * ex + ey * ey + ez * ez;
                    if (n2 > kMaxNorm2) continue;
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

template <int KIND>
inline constexpr Lattice<KIND> kLattice = Lattice<KIND>::make();

template <int KIND>
inline constexpr int kDim = Lattice<KIND>::D;

// Compile-time checks of the generated sets: opposite index, weights summing
// to one and the second moment c_s^2 = 1/3.
template <int KIND>
constexpr bool lattice_ok()
{
    constexpr auto L = kLattice<KIND>;
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
static_assert(lattice_ok<0>(), "D2Q9 table");
static_assert(lattice_ok<1>(), "D3Q19 table");
static_assert(lattice_ok<2>(), "D3Q27 table");
static_assert(kLattice<0>.e[0][0] == -1 && kLattice<0>.e[0][1] == -1 && kLattice<0>.e[4][0] == 0,
              "D2Q9 numbering of Sec. 2.1");
static_assert(kLattice<1>.e[9][0] == 0 && kLattice<1>.e[9][1] == 0 && kLattice<1>.e[9][2] == 0,
              "D3Q19 rest direction in the middle");
static_assert(kLattice<2>.e[13][0] == 0 && kLattice<2>.e[13][1] == 0 && kLattice<2>.e[13][2] == 0,
              "D3Q27 rest direction in the middle");

}  // namespace imexlbm
