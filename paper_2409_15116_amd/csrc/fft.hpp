// 3D FFT plans and sphere index maps.
#pragma once

#include "common.hpp"

namespace bse {

// FFT lengths compiled into the library (products of 2, 3 and 5)
#define BSE_FFT_SIZES(X) X(16) X(24) X(32) X(36) X(48) X(60) X(64) X(72) X(80) X(96) X(120) X(128)

struct FftPlan {
    int n;
    int nst;
    int radix[8];
};

// Device-resident index maps of the wavefunction sphere on an n^3 grid.
struct SphereMaps {
    int n = 0;
    int npw = 0;
    int ncol = 0;             // padded even column count (col 0 = (0,0), col 1 = empty)
    int nxp = 0;              // x-planes holding sphere points
    FftPlan plan{};
    int2 *ent = nullptr;      // per column: {z | kind << 16, packed index}
    int *col_ptr = nullptr;   // [ncol + 1]
    int *colmap = nullptr;    // [n * n] (x, y) -> column or -1
    int *xlist = nullptr;     // [nxp] grid x of each sphere plane
    int *xinv = nullptr;      // [n] grid x -> plane or -1
    double *kin = nullptr;    // [npw] 1/2 |G|^2 per packed dof
};

FftPlan make_plan(int n);

// ev (optional): three events recorded after the three passes.
// Two real orbitals share a complex transform: o and o + ps (ps = 1 pairs
// neighbours; ps = n_occ pairs the same slot of consecutive trial vectors,
// n_orb a multiple of ps).  Workspaces hold ceil(n_orb / 2ps) * ps lines.
template <typename T>
void sph_inverse(const SphereMaps &m, const T *X, int n_orb, T *out, cplx<T> *T1, cplx<T> *T2,
                 const cplx<T> *tw, hipStream_t st, hipEvent_t *ev = nullptr, int ps = 1);

// pairs the same orbital slot of consecutive trial vectors (ps = n_occ)
template <typename T>
void sph_forward(const SphereMaps &m, const T *Cr, const T *u, const cplx<T> *vH, T k1e, int n_orb,
                 int n_occ, const T *X, T kin_scale, T *Y, cplx<T> *T1, cplx<T> *T2,
                 const cplx<T> *tw, hipStream_t st, hipEvent_t *ev = nullptr);

template <typename T>
void grid_fft(const FftPlan &pl, cplx<T> *A, int nb, T sign, const cplx<T> *tw, hipStream_t st);

}  // namespace bse
