// Lattice tables for the HIP engine, built at compile time.
//
// D2Q9: velocity order and weights of the paper's Appendix (D2Q9 model);
// moment rows are the Lallemand-Luo polynomials 1, 3e^2-4,
// (9e^4-21e^2+8)/2, e_x, (3e^2-5)e_x, e_y, (3e^2-5)e_y, e_x^2-e_y^2, e_x e_y,
// which reproduce the matrix printed in the Appendix.
// D3Q15: velocity order, weights and transformation matrix of the paper's
// Appendix (D3Q15 model); its rows are the polynomials 1, e^2-2,
// (15e^4-55e^2+32)/2, e_a and (5e^2-13)e_a/2 for a = x, y, z, 3e_x^2-e^2,
// e_y^2-e_z^2, e_x e_y, e_y e_z, e_x e_z and e_x e_y e_z.
// D3Q19: rest, axis and edge vectors, weights 1/3, 1/18, 1/36; rows are the
// d'Humieres et al. (2002) moment polynomials (the reference the paper
// cites for its 3D MRT models).
// Everything here is constexpr so that, after unrolling, every multiply by
// a matrix entry is folded into an add, a subtract, a scaled FMA or nothing.
#pragma once

#include <cstdint>
#include <utility>

namespace lbe {

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr int E[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},
                                    {-1, 0, 0}, {0, -1, 0}, {1, 1, 0},
                                    {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    static constexpr double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr int moment(int k, int i) {
        const int ex = E[i][0], ey = E[i][1];
        const int e2 = ex * ex + ey * ey;
        switch (k) {
            case 0: return 1;
            case 1: return 3 * e2 - 4;
            case 2: return (9 * e2 * e2 - 21 * e2 + 8) / 2;
            case 3: return ex;
            case 4: return (3 * e2 - 5) * ex;
            case 5: return ey;
            case 6: return (3 * e2 - 5) * ey;
            case 7: return ex * ex - ey * ey;
            default: return ex * ey;
        }
    }
    // rows whose non-equilibrium part is identically zero (density, momentum)
    static constexpr bool conserved(int k) { return k == 0 || k == 3 || k == 5; }
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr int E[19][3] = {
        {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
        {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, 1, 0},  {1, -1, 0},
        {-1, -1, 0}, {1, 0, 1}, {-1, 0, 1}, {1, 0, -1},  {-1, 0, -1},
        {0, 1, 1},  {0, -1, 1}, {0, 1, -1}, {0, -1, -1}};
    static constexpr double W[19] = {
        1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr int moment(int k, int i) {
        const int ex = E[i][0], ey = E[i][1], ez = E[i][2];
        const int e2 = ex * ex + ey * ey + ez * ez;
        switch (k) {
            case 0: return 1;
            case 1: return 19 * e2 - 30;
            case 2: return (21 * e2 * e2 - 53 * e2 + 24) / 2;
            case 3: return ex;
            case 4: return (5 * e2 - 9) * ex;
            case 5: return ey;
            case 6: return (5 * e2 - 9) * ey;
            case 7: return ez;
            case 8: return (5 * e2 - 9) * ez;
            case 9: return 3 * ex * ex - e2;
            case 10: return (3 * e2 - 5) * (3 * ex * ex - e2);
            case 11: return ey * ey - ez * ez;
            case 12: return (3 * e2 - 5) * (ey * ey - ez * ez);
            case 13: return ex * ey;
            case 14: return ey * ez;
            case 15: return ex * ez;
            case 16: return (ey * ey - ez * ez) * ex;
            case 17: return (ez * ez - ex * ex) * ey;
            default: return (ex * ex - ey * ey) * ez;
        }
    }
    static constexpr bool conserved(int k) {
        return k == 0 || k == 3 || k == 5 || k == 7;
    }
};

struct D3Q15 {
    static constexpr int Q = 15;
    static constexpr int D = 3;
    static constexpr int E[15][3] = {
        {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
        {0, 0, 1},  {0, 0, -1},  {1, 1, 1},  {-1, 1, 1}, {1, -1, 1},
        {-1, -1, 1}, {1, 1, -1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};
    static constexpr double W[15] = {2.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9,
                                     1.0 / 9,  1.0 / 9,  1.0 / 72, 1.0 / 72, 1.0 / 72,
                                     1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72};
    static constexpr int moment(int k, int i) {
        const int ex = E[i][0], ey = E[i][1], ez = E[i][2];
        const int e2 = ex * ex + ey * ey + ez * ez;
        switch (k) {
            case 0: return 1;
            case 1: return e2 - 2;
            case 2: return (15 * e2 * e2 - 55 * e2 + 32) / 2;
            case 3: return ex;
            case 4: return (5 * e2 - 13) * ex / 2;
            case 5: return ey;
            case 6: return (5 * e2 - 13) * ey / 2;
            case 7: return ez;
            case 8: return (5 * e2 - 13) * ez / 2;
            case 9: return 3 * ex * ex - e2;
            case 10: return ey * ey - ez * ez;
            case 11: return ex * ey;
            case 12: return ey * ez;
            case 13: return ex * ez;
            default: return ex * ey * ez;
        }
    }
    static constexpr bool conserved(int k) {
        return k == 0 || k == 3 || k == 5 || k == 7;
    }
};

template <class L>
struct Tables {
    int M[L::Q][L::Q];
    int norm[L::Q];
    int opp[L::Q];
    constexpr Tables() : M(), norm(), opp() {
        for (int k = 0; k < L::Q; ++k) {
            int s = 0;
            for (int i = 0; i < L::Q; ++i) {
                M[k][i] = L::moment(k, i);
                s += M[k][i] * M[k][i];
            }
            norm[k] = s;
        }
        for (int i = 0; i < L::Q; ++i)
            for (int j = 0; j < L::Q; ++j)
                if (L::E[j][0] == -L::E[i][0] && L::E[j][1] == -L::E[i][1] &&
                    L::E[j][2] == -L::E[i][2])
                    opp[i] = j;
    }
};

template <class L>
inline constexpr Tables<L> TAB{};

// Quantities derived from the tables for the symmetric form of the MRT
// transform.  Velocities come in opposite pairs (i, ibar); every moment row
// is either even (M_k,ibar = M_k,i) or odd (M_k,ibar = -M_k,i), so with
// s_p = f_i + f_ibar and d_p = f_i - f_ibar an even row needs only f_0 and
// the s_p, an odd row only the d_p.  The equilibrium moments are written in
// closed form, m^eq_k = A_k drho + B_k.j + sum_c C_kc (jj)_c / rho0, where
// (jj) = (jx^2, jy^2, jz^2, jx jy, jy jz, jx jz), by projecting Eq. (42)
// onto the rows: A_k = sum_i M_ki w_i, B_ka = 3 sum_i M_ki w_i e_ia and
// C_kab = 4.5 sum_i M_ki w_i e_ia e_ib - 1.5 delta_ab A_k (doubled for a != b).
template <class L>
struct Derived {
    int npair;
    int pi[(L::Q - 1) / 2];     // the member i of each pair with i < ibar
    bool even[L::Q];
    double A[L::Q];
    double B[L::Q][3];
    double C[L::Q][6];
    constexpr Derived() : npair(0), pi(), even(), A(), B(), C() {
        const auto& t = TAB<L>;
        for (int i = 1; i < L::Q; ++i)
            if (t.opp[i] > i) pi[npair++] = i;
        for (int k = 0; k < L::Q; ++k) {
            even[k] = true;
            for (int i = 0; i < L::Q; ++i)
                if (t.M[k][t.opp[i]] != t.M[k][i]) even[k] = false;
            double a = 0, b[3] = {0, 0, 0}, c[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int i = 0; i < L::Q; ++i) {
                const double mw = t.M[k][i] * L::W[i];
                a += mw;
                for (int x = 0; x < 3; ++x) {
                    b[x] += 3.0 * mw * L::E[i][x];
                    for (int y = 0; y < 3; ++y) c[x][y] += 4.5 * mw * L::E[i][x] * L::E[i][y];
                }
            }
            A[k] = a;
            for (int x = 0; x < 3; ++x) B[k][x] = b[x];
            C[k][0] = c[0][0] - 1.5 * a;
            C[k][1] = c[1][1] - 1.5 * a;
            C[k][2] = c[2][2] - 1.5 * a;
            C[k][3] = 2.0 * c[0][1];
            C[k][4] = 2.0 * c[1][2];
            C[k][5] = 2.0 * c[0][2];
        }
    }
};

template <class L>
inline constexpr Derived<L> DER{};

// every row is even or odd, and the conserved rows are density and momentum
template <class L>
constexpr bool rows_have_parity() {
    for (int k = 0; k < L::Q; ++k) {
        bool ev = true, od = true;
        for (int i = 0; i < L::Q; ++i) {
            if (TAB<L>.M[k][TAB<L>.opp[i]] != TAB<L>.M[k][i]) ev = false;
            if (TAB<L>.M[k][TAB<L>.opp[i]] != -TAB<L>.M[k][i]) od = false;
        }
        if (ev == od) return false;
    }
    return DER<L>.npair * 2 + 1 == L::Q;
}
static_assert(rows_have_parity<D2Q9>(), "D2Q9 rows must be even or odd");
static_assert(rows_have_parity<D3Q19>(), "D3Q19 rows must be even or odd");
static_assert(rows_have_parity<D3Q15>(), "D3Q15 rows must be even or odd");

// the printed D3Q15 matrix: spot checks of rows 2, 4 and 14 (0-based)
static_assert(TAB<D3Q15>.M[2][0] == 16 && TAB<D3Q15>.M[2][1] == -4 && TAB<D3Q15>.M[2][7] == 1,
              "D3Q15 row 2");
static_assert(TAB<D3Q15>.M[4][1] == -4 && TAB<D3Q15>.M[4][2] == 4 && TAB<D3Q15>.M[4][8] == -1,
              "D3Q15 row 4");
static_assert(TAB<D3Q15>.M[14][7] == 1 && TAB<D3Q15>.M[14][8] == -1 && TAB<D3Q15>.M[14][11] == -1,
              "D3Q15 row 14");

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1.
template <class F, int... I>
__host__ __device__ __forceinline__ void unroll_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void unroll(F&& f) {
    unroll_impl(f, std::make_integer_sequence<int, N>{});
}

}  // namespace lbe
