// Device kernels of the single-level spectral Ewald variant (periodic unit
// cell, uniform data): spreading to an M^3 grid, Fourier-space scaling and
// interpolation back to the points (Sec. "Ewald summation": spread, FFT,
// scale, inverse FFT, interpolate).  The near field reuses the DMK residual
// kernel between cells of the split level.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmk {

// Gridding kernel g(t) = sum_k a_k T_k(2 t^2 - 1) for |t| < 1, 0 outside
// (t = (X - n) / (w/2) in grid units).
constexpr int kGridTerms = 24;
struct GridPoly {
    int nc;                 // terms in use (<= kGridTerms); the rest are zero
    double a[kGridTerms];
};

// Tiles are the Morton cells of level Lt (side B grid points, M = B 2^Lt):
// tile t holds the sorted points [tile_start[t], tile_start[t+1]).
// Points are the sorted centred unit-cell coordinates x, y, z in [-1/2, 1/2)
// (grid coordinate X = (x + 1/2) M).

// grid[c][ix][iy][iz] (M^3 reals per component c) = sum_s fs[c][s] g_x g_y g_z
// over the w-point stencil of every point image; every grid value is written
// once by the block of its tile (a deterministic gather, no atomics).
void launch_ewald_spread(int M, int B, int Lt, int w, const GridPoly& g, const int64_t* tile_start, const double* x,
                         const double* y, const double* z, const double* fs, int64_t n, double* grid,
                         hipStream_t s);

// In place on the half spectrum spec[c][i][j][k] (M x M x (M/2+1) complex per
// component, the layout of a 3D real-to-complex FFT): for 0 < |kappa|,
// |kappa_i| <= K,  U = wsym(|kappa|^2) / (ghat_x ghat_y ghat_z)^2 (I - k k^T/k^2) F,
// and 0 elsewhere.
void launch_ewald_scale(int M, int K, const double* ghat, const double* wsym, double2* spec, hipStream_t s);

// u[c][i] = sum over the stencil of g_x g_y g_z grid[c][..] for every sorted
// point i (overwrites u); w in {6, 8, 11}.
void launch_ewald_interp(int M, int B, int Lt, int w, const GridPoly& g, const int64_t* tile_start,
                         const double* x, const double* y, const double* z, int64_t n, const double* grid,
                         double* u, hipStream_t s);

}  // namespace dmk
