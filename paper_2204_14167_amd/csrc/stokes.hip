// Overdamped Stokes with no-slip walls on the MAC grid (eq disc_stokes, eq fluidbc,
// eq disc_stokes_temp), hydrodynamic spreading S^hy and interpolation J^hy
// (eq kernel2, eq kernel1, Fig. folded, ghost rule for interpolation).
//
// Mode solve: after the in-plane FFTs, each mode (m, n) with kappa != 0 is rotated
// onto e = (G_x, G_y) / kappa, G the symbols of the face gradient:
//   b = e_perp^H u   obeys eta T b = f_perp            (T = -D_zz + kappa^2, walls),
//   a = e^H u, w, p  obey  eta T a + kappa p = f_par,  eta T_w w + G_z p = f_z,
//                          -kappa a + D_z w = 0,
// a real 3x3 block-tridiagonal saddle system in z solved by block Thomas (one thread
// per mode).  kappa = 0: tridiagonal solves for the mean flow, w = 0, the pressure
// from its z-gradient with mean zero.
#include "kernels.h"

namespace discos {

// ---- S^hy: force spreading on one face grid (tile gather, as the charge spread) ----
#define SH_TX 16
#define SH_THREADS 256
#define SH_MAXR 256

// Deposit val * phi(x - node) / h^3 of one kernel centre (px, py, pz) into the tile.
// COMP 0 / 1: x / y component at cell-centre heights, images fold k -> -1-k with the
// wall's tangential sign g.tsg (-1 no-slip, +1 slip).  COMP 2: z component on z-faces,
// images fold k -> -k (sign -1); wall faces hold 0.
template <int COMP>
__device__ __forceinline__ void deposit_face(const GridDev& g, double* acc, int x0, int y0, int z0,
                                             int tx, int ty, int tz, double px, double py,
                                             double pz, double val) {
    const double ox = COMP == 0 ? 0.0 : 0.5, oy = COMP == 1 ? 0.0 : 0.5, oz = COMP == 2 ? 0.0 : 0.5;
    int ix0, iy0, iz0;
    double wx[4], wy[4], wz[4];
    peskin4(px * g.inv_h - ox, ix0, wx);
    peskin4(py * g.inv_h - oy, iy0, wy);
    peskin4(pz * g.inv_h - oz, iz0, wz);
    int lxs[4], lys[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) lxs[a] = (ix0 + a - x0) & (g.nx - 1);
#pragma unroll
    for (int b = 0; b < 4; ++b) lys[b] = (iy0 + b - y0) & (g.ny - 1);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int kz = iz0 + c;
        double sgn = 1.0;
        if (COMP == 2) {
            if (kz < 0) { kz = -kz; sgn = -1.0; }
            else if (kz > g.nz) { kz = 2 * g.nz - kz; sgn = -1.0; }
            if (kz == 0 || kz == g.nz) continue;
        } else {
            if (kz < 0) { kz = -1 - kz; sgn = g.tsg[0]; }
            else if (kz >= g.nz) { kz = 2 * g.nz - 1 - kz; sgn = g.tsg[1]; }
        }
        const int lz = kz - z0;
        if (lz < 0 || lz >= tz) continue;
        const double wzc = val * sgn * wz[c];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (lys[b] >= ty) continue;
            const double wyz = wzc * wy[b];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (lxs[a] >= tx) continue;
                atomicAdd(&acc[(lz * ty + lys[b]) * tx + lxs[a]], wyz * wx[a]);
            }
        }
    }
}

// ---- hydrodynamic kernels per species (App. B, eq eskernel) ----------------------
// Row of the kernel table for species sp: (w, beta, 1 / alpha, 1 / integral); species
// outside [0, DISCOS_HY_MAXSP) use the extra last row, always the 4-point Peskin kernel
// (w = 0), as do the species past the ones set.
__device__ __forceinline__ const double* hy_row(const double* __restrict__ tab, int sp) {
    return tab + 4 * ((sp >= 0 && sp < DISCOS_HY_MAXSP) ? sp : DISCOS_HY_MAXSP);
}

// phi(zeta), zeta in cells: the 4-point Peskin kernel of eq peskin1d for w = 0, else
// the ESC kernel exp(beta (sqrt(1 - (zeta / alpha)^2) - 1)) / integral, zero from
// |zeta| = alpha = w / 2 on.
__device__ __forceinline__ double hy_weight(double zeta, double w, double beta, double inv_alpha,
                                           double inv_norm) {
    const double r = fabs(zeta);
    if (w == 0.0) {
        if (r < 1.0) return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) * 0.125;
        if (r < 2.0) return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) * 0.125;
        return 0.0;
    }
    if (r < 0.5 * w) {
        const double t = zeta * inv_alpha;
        return exp(beta * (sqrt(fmax(1.0 - t * t, 0.0)) - 1.0)) * inv_norm;
    }
    return 0.0;
}

// Weights of the 2 KM nodes floor(s) + 1 - KM + a, a = 0 .. 2 KM - 1, of one axis (zero
// outside the kernel's support); returns the first node.
template <int KM>
__device__ __forceinline__ int hy_axis(double s, const double* kr, double* wt) {
    const double fl = floor(s);
    const int i0 = (int)fl + 1 - KM;
#pragma unroll
    for (int a = 0; a < 2 * KM; ++a)
        wt[a] = hy_weight(s - (double)(i0 + a), kr[0], kr[1], kr[2], kr[3]);
    return i0;
}

// The force deposit v0 phi(x - node) and the random finite difference
// v [phi(x + d - node) - phi(x - d - node)] of one ion in one pass, one atomic per node:
// possible when the three kernel centres' windows start at the same node on every axis
// (the shift d is far below a cell, so nearly always).  Returns false, depositing
// nothing, otherwise.  Folds as deposit_face.
template <int COMP>
__device__ __forceinline__ bool deposit_face_rfd(const GridDev& g, double* acc, int x0, int y0,
                                                 int z0, int tx, int ty, int tz, double px,
                                                 double py, double pz, double hx, double hy,
                                                 double hz, double v0, double v) {
    const double ox = COMP == 0 ? 0.0 : 0.5, oy = COMP == 1 ? 0.0 : 0.5, oz = COMP == 2 ? 0.0 : 0.5;
    int ix0, iy0, iz0, jx, jy, jz, kx, ky, kz;
    double wx0[4], wxp[4], wxm[4], wy0[4], wyp[4], wym[4], wz0[4], wzp[4], wzm[4];
    peskin4(px * g.inv_h - ox, ix0, wx0);
    peskin4((px + hx) * g.inv_h - ox, jx, wxp);
    peskin4((px - hx) * g.inv_h - ox, kx, wxm);
    peskin4(py * g.inv_h - oy, iy0, wy0);
    peskin4((py + hy) * g.inv_h - oy, jy, wyp);
    peskin4((py - hy) * g.inv_h - oy, ky, wym);
    peskin4(pz * g.inv_h - oz, iz0, wz0);
    peskin4((pz + hz) * g.inv_h - oz, jz, wzp);
    peskin4((pz - hz) * g.inv_h - oz, kz, wzm);
    if (jx != ix0 || kx != ix0 || jy != iy0 || ky != iy0 || jz != iz0 || kz != iz0) return false;
    int lxs[4], lys[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) lxs[a] = (ix0 + a - x0) & (g.nx - 1);
#pragma unroll
    for (int b = 0; b < 4; ++b) lys[b] = (iy0 + b - y0) & (g.ny - 1);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int kk = iz0 + c;
        double sgn = 1.0;
        if (COMP == 2) {
            if (kk < 0) { kk = -kk; sgn = -1.0; }
            else if (kk > g.nz) { kk = 2 * g.nz - kk; sgn = -1.0; }
            if (kk == 0 || kk == g.nz) continue;
        } else {
            if (kk < 0) { kk = -1 - kk; sgn = g.tsg[0]; }
            else if (kk >= g.nz) { kk = 2 * g.nz - 1 - kk; sgn = g.tsg[1]; }
        }
        const int lz = kk - z0;
        if (lz < 0 || lz >= tz) continue;
        const double z0c = sgn * v0 * wz0[c], zpc = sgn * v * wzp[c], zmc = sgn * v * wzm[c];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (lys[b] >= ty) continue;
            const double y0c = z0c * wy0[b], ypc = zpc * wyp[b], ymc = zmc * wym[b];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                if (lxs[a] >= tx) continue;
                atomicAdd(&acc[(lz * ty + lys[b]) * tx + lxs[a]],
                          y0c * wx0[a] + (ypc * wxp[a] - ymc * wxm[a]));
            }
        }
    }
    return true;
}

// S^hy F on one face grid with the 4-point Peskin kernel; with rfd.scale != 0 every ion
// also deposits the random finite difference (kT / delta) [phi(x + delta/2 W) -
// phi(x - delta/2 W)] W_COMP of the thermal forcing.  The shifts are below half a cell:
// along an axis whose nodes sit on faces, a kernel shifted up from the cell below the
// tile's two-cell window reaches the tile's first node, so the candidate rows then reach
// three cells down.
template <int COMP, int T>
__global__ void __launch_bounds__(SH_THREADS)
spread_face_kernel(GridDev g, const double4* __restrict__ sxyzq, const double* __restrict__ fw,
                   const int* __restrict__ bin_start, RfdDev rfd, double* __restrict__ out,
                   int* __restrict__ flags) {
    __shared__ double acc[T * T * T];
    __shared__ int rstart[SH_MAXR], rpre[SH_MAXR + 1], scan[SH_THREADS];
    const int nzn = COMP == 2 ? g.nz + 1 : g.nz;  // node levels
    const int tx = min(T, g.nx), ty = min(T, g.ny);
    const int x0 = blockIdx.x * tx, y0 = blockIdx.y * ty, z0 = blockIdx.z * T;
    const int tz = min(T, nzn - z0);
    const int ncell = tx * ty * tz;
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) acc[k] = 0.0;
    // ions that can reach node levels [z0, z0+tz): cells [z0-2, z0+tz+1] (one more below
    // with the shifts)
    static_assert(tile_rows_bound(T, T, 3, 2) <= SH_MAXR, "face spread tile rows exceed SH_MAXR");
    const int nr = tile_ranges<SH_MAXR>(g, bin_start, x0, y0, z0, tx, ty, min(tz, g.nz - z0 + 1),
                                        rstart, rpre, scan, flags, rfd.scale != 0.0 ? 3 : 2, 2);
    const int total = rpre[nr];
    const double inv_h3 = g.inv_h * g.inv_h * g.inv_h;
    for (int f = threadIdx.x; f < total; f += blockDim.x) {
        int r = 0, hi = nr - 1;
        while (r < hi) {
            const int mid = (r + hi + 1) >> 1;
            if (rpre[mid] <= f) r = mid; else hi = mid - 1;
        }
        const int i = rstart[r] + (f - rpre[r]);
        const double4 a4 = sxyzq[i];
        if (!pos_ok(g, a4.x, a4.y, a4.z)) continue;
        const double v0 = fw[i] * inv_h3;
        if (rfd.scale == 0.0) {
            deposit_face<COMP>(g, acc, x0, y0, z0, tx, ty, tz, a4.x, a4.y, a4.z, v0);
            continue;
        }
        const double w0 = rfd.w[i], w1 = rfd.w[i + rfd.wstride], w2 = rfd.w[i + 2 * rfd.wstride];
        const double wc = COMP == 0 ? w0 : (COMP == 1 ? w1 : w2);
        const double v = rfd.scale * wc * inv_h3;
        const double hx = rfd.half * w0, hy = rfd.half * w1, hz = rfd.half * w2;
        if (deposit_face_rfd<COMP>(g, acc, x0, y0, z0, tx, ty, tz, a4.x, a4.y, a4.z, hx, hy, hz, v0, v))
            continue;
        deposit_face<COMP>(g, acc, x0, y0, z0, tx, ty, tz, a4.x, a4.y, a4.z, v0);
        deposit_face<COMP>(g, acc, x0, y0, z0, tx, ty, tz, a4.x + hx, a4.y + hy, a4.z + hz, v);
        deposit_face<COMP>(g, acc, x0, y0, z0, tx, ty, tz, a4.x - hx, a4.y - hy, a4.z - hz, -v);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int lx = k % tx, ly = (k / tx) % ty, lz = k / (tx * ty);
        const int gk = z0 + lz;
        double v = acc[k];
        if (COMP == 2 && (gk == 0 || gk == g.nz)) v = 0.0;
        out[((size_t)gk * g.ny + (y0 + ly)) * g.nx + (x0 + lx)] = v;
    }
}

// The random finite difference's normals W of every ion (keyed by its stable id),
// drawn once for the three component spreads.
__global__ void rfd_normals_kernel(int n, const int* __restrict__ sid, uint64_t seed, uint64_t step,
                                   double* __restrict__ w, int64_t stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double w0, w1, w2, unused;
    const uint32_t idi = (uint32_t)sid[i];
    normal_pair(seed, step, DISCOS_TAG_RFD, 0u, idi, w0, w1);
    normal_pair(seed, step, DISCOS_TAG_RFD, 1u, idi, w2, unused);
    w[i] = w0;
    w[i + stride] = w1;
    w[i + 2 * stride] = w2;
}

// ---- table kernels: each ion visited once ----------------------------------------------
// A table kernel's window of 2 KM nodes per axis reaches over several tiles, so a spread
// that lets every tile gather the ions of its halo evaluates an ion's weights once per
// tile it reaches (about 3.4 tiles per component for 8-node windows on 16^3 tiles), and
// every node test is repeated with them.  Here a tile takes only the ions of its own
// cells and deposits their whole windows into an LDS region of the tile's nodes plus
// own_h(KM) = KM + 1 nodes on every side, which holds the window of any ion of the tile
// and of its two random-finite-difference shifts and, after the one fold at a wall, every
// image level.  (A shift is delta/2 |W| with delta <= 0.1 h and |W| <= 8.6 for normals
// drawn from 53-bit uniforms, so below half a cell: a window's first node moves by at
// most one.)  The
// region is then added to the grid (zeroed beforehand) with global atomics, consecutive
// lanes on consecutive x nodes.  Each ion's weights are evaluated once per axis.
#define OWN_T 16
#define OWN_THREADS 512
#define OWN_MAXR 128  // bin rows of a 16^3 tile: 8 x 8, bounded as if each had two x segments
constexpr int own_h(int KM) { return KM + 1; }
constexpr int own_e(int KM) { return OWN_T + 2 * own_h(KM); }

// Weights of one axis at the nodes i0 .. i0 + 2 KM - 1 (i0 = floor(s) + 1 - KM).
template <int KM>
__device__ __forceinline__ void own_axis(double s, int i0, const double* kr, double* wt) {
#pragma unroll
    for (int a = 0; a < 2 * KM; ++a) wt[a] = hy_weight(s - (double)(i0 + a), kr[0], kr[1], kr[2], kr[3]);
}

// Local level of node level kz after the one fold at a wall, and the fold's sign;
// false for a wall face of the z component (it carries nothing).
template <int COMP>
__device__ __forceinline__ bool own_level(const GridDev& g, int kz, int oz, int& lz, double& sgn) {
    sgn = 1.0;
    if (COMP == 2) {
        if (kz < 0) { kz = -kz; sgn = -1.0; }
        else if (kz > g.nz) { kz = 2 * g.nz - kz; sgn = -1.0; }
        if (kz == 0 || kz == g.nz) return false;
    } else {
        if (kz < 0) { kz = -1 - kz; sgn = g.tsg[0]; }
        else if (kz >= g.nz) { kz = 2 * g.nz - 1 - kz; sgn = g.tsg[1]; }
    }
    lz = kz - oz;
    return true;
}

// v phi(x - node) of one kernel centre into the region (origin ox, oy, oz; rows of ex,
// planes of exy doubles).
template <int COMP, int KM>
__device__ __forceinline__ void own_deposit1(const GridDev& g, double* acc, int ox, int oy, int oz,
                                             int ex, int exy, double px, double py, double pz,
                                             double v, const double* kr) {
    constexpr int NW = 2 * KM;
    const double sx = px * g.inv_h - (COMP == 0 ? 0.0 : 0.5);
    const double sy = py * g.inv_h - (COMP == 1 ? 0.0 : 0.5);
    const double sz = pz * g.inv_h - (COMP == 2 ? 0.0 : 0.5);
    const int ix0 = (int)floor(sx) + 1 - KM, iy0 = (int)floor(sy) + 1 - KM, iz0 = (int)floor(sz) + 1 - KM;
    double wx[NW], wy[NW];
    own_axis<KM>(sx, ix0, kr, wx);
    own_axis<KM>(sy, iy0, kr, wy);
    const int lx = ix0 - ox, ly = iy0 - oy;
    for (int c = 0; c < NW; ++c) {
        int lz;
        double sgn;
        if (!own_level<COMP>(g, iz0 + c, oz, lz, sgn)) continue;
        const double wz = hy_weight(sz - (double)(iz0 + c), kr[0], kr[1], kr[2], kr[3]);
        if (wz == 0.0) continue;
        const double wzc = v * sgn * wz;
        double* plane = acc + lz * exy + ly * ex + lx;
        // every node of the level, zero weights included: a branch per node costs more
        // than the atomic it would save
#pragma unroll
        for (int b = 0; b < NW; ++b) {
            const double wyz = wzc * wy[b];
#pragma unroll
            for (int a = 0; a < NW; ++a) atomicAdd(&plane[b * ex + a], wyz * wx[a]);
        }
    }
}

// The force v0 phi(x - node) and the random finite difference v [phi(x + d - node) -
// phi(x - d - node)] of one ion in one pass (one atomic per node) when the three
// windows start at the same node on every axis; false (nothing deposited) otherwise.
template <int COMP, int KM>
__device__ __forceinline__ bool own_deposit_rfd(const GridDev& g, double* acc, int ox, int oy, int oz,
                                                int ex, int exy, double px, double py, double pz,
                                                double hx, double hy, double hz, double v0, double v,
                                                const double* kr) {
    constexpr int NW = 2 * KM;
    const double ofx = COMP == 0 ? 0.0 : 0.5, ofy = COMP == 1 ? 0.0 : 0.5, ofz = COMP == 2 ? 0.0 : 0.5;
    const double sx = px * g.inv_h - ofx, sy = py * g.inv_h - ofy, sz = pz * g.inv_h - ofz;
    const double sxp = (px + hx) * g.inv_h - ofx, syp = (py + hy) * g.inv_h - ofy,
                 szp = (pz + hz) * g.inv_h - ofz;
    const double sxm = (px - hx) * g.inv_h - ofx, sym = (py - hy) * g.inv_h - ofy,
                 szm = (pz - hz) * g.inv_h - ofz;
    const double fx = floor(sx), fy = floor(sy), fz = floor(sz);
    if (floor(sxp) != fx || floor(sxm) != fx || floor(syp) != fy || floor(sym) != fy ||
        floor(szp) != fz || floor(szm) != fz)
        return false;
    const int ix0 = (int)fx + 1 - KM, iy0 = (int)fy + 1 - KM, iz0 = (int)fz + 1 - KM;
    double wx0[NW], wxp[NW], wxm[NW], wy0[NW], wyp[NW], wym[NW];
    own_axis<KM>(sx, ix0, kr, wx0);
    own_axis<KM>(sxp, ix0, kr, wxp);
    own_axis<KM>(sxm, ix0, kr, wxm);
    own_axis<KM>(sy, iy0, kr, wy0);
    own_axis<KM>(syp, iy0, kr, wyp);
    own_axis<KM>(sym, iy0, kr, wym);
    const int lx = ix0 - ox, ly = iy0 - oy;
    for (int c = 0; c < NW; ++c) {
        int lz;
        double sgn;
        if (!own_level<COMP>(g, iz0 + c, oz, lz, sgn)) continue;
        const double nz = (double)(iz0 + c);
        double z0c = hy_weight(sz - nz, kr[0], kr[1], kr[2], kr[3]);
        double zpc = hy_weight(szp - nz, kr[0], kr[1], kr[2], kr[3]);
        double zmc = hy_weight(szm - nz, kr[0], kr[1], kr[2], kr[3]);
        if (z0c == 0.0 && zpc == 0.0 && zmc == 0.0) continue;
        z0c *= sgn * v0;
        zpc *= sgn * v;
        zmc *= sgn * v;
        double* plane = acc + lz * exy + ly * ex + lx;
#pragma unroll
        for (int b = 0; b < NW; ++b) {
            const double y0c = z0c * wy0[b], ypc = zpc * wyp[b], ymc = zmc * wym[b];
#pragma unroll
            for (int a = 0; a < NW; ++a)
                atomicAdd(&plane[b * ex + a], y0c * wx0[a] + (ypc * wxp[a] - ymc * wxm[a]));
        }
    }
    return true;
}

// One ion's deposits: the force, and with rfd its random finite difference (merged when
// the three windows coincide, else three deposits).
template <int COMP, int KM>
__device__ __forceinline__ void own_ion(const GridDev& g, double* acc, int ox, int oy, int oz, int ex,
                                        int exy, double4 a4, bool rfd, double hx, double hy, double hz,
                                        double v0, double v, const double* kr) {
    if (!rfd) {
        own_deposit1<COMP, KM>(g, acc, ox, oy, oz, ex, exy, a4.x, a4.y, a4.z, v0, kr);
        return;
    }
    if (own_deposit_rfd<COMP, KM>(g, acc, ox, oy, oz, ex, exy, a4.x, a4.y, a4.z, hx, hy, hz, v0, v, kr))
        return;
    own_deposit1<COMP, KM>(g, acc, ox, oy, oz, ex, exy, a4.x, a4.y, a4.z, v0, kr);
    own_deposit1<COMP, KM>(g, acc, ox, oy, oz, ex, exy, a4.x + hx, a4.y + hy, a4.z + hz, v, kr);
    own_deposit1<COMP, KM>(g, acc, ox, oy, oz, ex, exy, a4.x - hx, a4.y - hy, a4.z - hz, -v, kr);
}

// S^hy F (+ the random finite difference) of the table kernels on one face grid: tile
// (bx, by, bz) of OWN_T^3 cells takes the ions of its cells and adds its region to out,
// which the caller has zeroed.
template <int COMP, int KM>
__global__ void __launch_bounds__(OWN_THREADS)
spread_face_own_kernel(GridDev g, const double4* __restrict__ sxyzq, const double* __restrict__ fw,
                       const int* __restrict__ bin_start, RfdDev rfd, const int* __restrict__ ssp,
                       const double* __restrict__ hy_tab, double* __restrict__ out,
                       int* __restrict__ flags) {
    constexpr int H = own_h(KM), E = own_e(KM);
    __shared__ double acc[E * E * E];
    __shared__ int rstart[OWN_MAXR], rpre[OWN_MAXR + 1], scan[OWN_THREADS];
    static_assert(tile_rows_bound(OWN_T, OWN_T, 0, 0) <= OWN_MAXR, "own-tile rows exceed OWN_MAXR");
    int bx, by, bz;
    xcd_block3(bx, by, bz);
    const int tx = min(OWN_T, g.nx), ty = min(OWN_T, g.ny);
    const int x0 = bx * tx, y0 = by * ty, z0 = bz * OWN_T;
    const int tz = min(OWN_T, g.nz - z0);  // cells
    const int ex = tx + 2 * H, ey = ty + 2 * H, ez = tz + 2 * H;
    const int exy = ex * ey, ne = exy * ez;
    const int ox = x0 - H, oy = y0 - H, oz = z0 - H;
    for (int k = threadIdx.x; k < ne; k += OWN_THREADS) acc[k] = 0.0;
    const int nr = tile_ranges<OWN_MAXR>(g, bin_start, x0, y0, z0, tx, ty, tz, rstart, rpre, scan,
                                         flags, 0, 0);
    const int total = rpre[nr];
    const double inv_h3 = g.inv_h * g.inv_h * g.inv_h;
    for (int f = threadIdx.x; f < total; f += OWN_THREADS) {
        int r = 0, hi = nr - 1;
        while (r < hi) {
            const int mid = (r + hi + 1) >> 1;
            if (rpre[mid] <= f) r = mid; else hi = mid - 1;
        }
        const int i = rstart[r] + (f - rpre[r]);
        const double4 a4 = sxyzq[i];
        if (!pos_ok(g, a4.x, a4.y, a4.z)) continue;
        const double* row = hy_row(hy_tab, ssp[i]);
        const double kr[4] = {row[0], row[1], row[2], row[3]};
        const double v0 = fw[i] * inv_h3;
        double v = 0.0, hx = 0.0, hy = 0.0, hz = 0.0;
        if (rfd.scale != 0.0) {
            const double w0 = rfd.w[i], w1 = rfd.w[i + rfd.wstride], w2 = rfd.w[i + 2 * rfd.wstride];
            v = rfd.scale * (COMP == 0 ? w0 : (COMP == 1 ? w1 : w2)) * inv_h3;
            hx = rfd.half * w0;
            hy = rfd.half * w1;
            hz = rfd.half * w2;
        }
        own_ion<COMP, KM>(g, acc, ox, oy, oz, ex, exy, a4, rfd.scale != 0.0, hx, hy, hz, v0, v, kr);
    }
    __syncthreads();
    const int nzn = COMP == 2 ? g.nz + 1 : g.nz;  // node levels
    for (int k = threadIdx.x; k < ne; k += OWN_THREADS) {
        const double v = acc[k];
        if (v == 0.0) continue;
        const int lx = k % ex, ly = (k / ex) % ey, gz = oz + k / exy;
        if (gz < 0 || gz >= nzn) continue;  // never reached by a deposit (folded first)
        const int gx = wrapi(ox + lx, g.nx), gy = wrapi(oy + ly, g.ny);
        atomicAdd(&out[((size_t)gz * g.ny + gy) * g.nx + gx], v);
    }
}

template <int KM>
static void spread_faces_own(Ctx* c, const RfdDev& rfd, const int* ssp, double* out, hipStream_t s) {
    const GridDev& g = c->gd;
    const size_t ncell = (size_t)g.nx * g.ny * g.nz;
    fill_f64(out, 3 * (int64_t)ncell + (int64_t)g.nx * g.ny, 0.0, s);
    const int tx = std::min(OWN_T, g.nx), ty = std::min(OWN_T, g.ny);
    dim3 grid(g.nx / tx, g.ny / ty, (g.nz + OWN_T - 1) / OWN_T);
    spread_face_own_kernel<0, KM><<<grid, OWN_THREADS, 0, s>>>(g, c->sxyzq, c->fp, c->bin_start, rfd,
                                                              ssp, c->hy_tab, out, c->flags);
    spread_face_own_kernel<1, KM><<<grid, OWN_THREADS, 0, s>>>(g, c->sxyzq, c->fp + c->n_max,
                                                              c->bin_start, rfd, ssp, c->hy_tab,
                                                              out + ncell, c->flags);
    spread_face_own_kernel<2, KM><<<grid, OWN_THREADS, 0, s>>>(g, c->sxyzq, c->fp + 2 * c->n_max,
                                                              c->bin_start, rfd, ssp, c->hy_tab,
                                                              out + 2 * ncell, c->flags);
}

template <int T>
static void spread_faces(Ctx* c, const RfdDev& rfd, double* out, hipStream_t s) {
    const GridDev& g = c->gd;
    const int tx = std::min(T, g.nx), ty = std::min(T, g.ny);
    const size_t ncell = (size_t)g.nx * g.ny * g.nz;
    dim3 grid_c(g.nx / tx, g.ny / ty, (g.nz + T - 1) / T);
    dim3 grid_f(g.nx / tx, g.ny / ty, (g.nz + 1 + T - 1) / T);
    spread_face_kernel<0, T><<<grid_c, SH_THREADS, 0, s>>>(g, c->sxyzq, c->fp, c->bin_start, rfd, out,
                                                          c->flags);
    spread_face_kernel<1, T><<<grid_c, SH_THREADS, 0, s>>>(g, c->sxyzq, c->fp + c->n_max, c->bin_start,
                                                          rfd, out + ncell, c->flags);
    spread_face_kernel<2, T><<<grid_f, SH_THREADS, 0, s>>>(g, c->sxyzq, c->fp + 2 * c->n_max,
                                                          c->bin_start, rfd, out + 2 * ncell, c->flags);
}

int spread_force_sorted(Ctx* c, double* out, hipStream_t s, const RfdDev* rfd_in, int species, int n) {
    RfdDev rfd{};
    if (rfd_in) {
        rfd = *rfd_in;
        // the normals go to c->hvi, which the wet step fills only after the solve
        if (n > 0)
            rfd_normals_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, rfd.sid, rfd.seed, rfd.step, c->hvi,
                                                              c->n_max);
        rfd.w = c->hvi;
        rfd.wstride = c->n_max;
    }
    const int km = species ? c->hy_km : 0;
    if (km == 0) spread_faces<SH_TX>(c, rfd, out, s);
    else if (km <= 2) spread_faces_own<2>(c, rfd, c->ssp, out, s);
    else spread_faces_own<4>(c, rfd, c->ssp, out, s);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

// ---- stochastic stress --------------------------------------------------------
// Unit normals (Philox, counters as in the oracle): diagonal tag, cell index
// (pair 0 -> xx, yy; pair 1 -> zz); edge tag, z-level index (k ny + j) nx + i with
// k = 0..nz (pair 0 -> xz, yz; pair 1 -> xy for k < nz).  Z_aa = sqrt(2) W, Z_ab = W,
// and the xz / yz edges on the walls (k = 0, nz) carry sqrt(2) W.
__global__ void stress_kernel(GridDev g, uint64_t seed, uint64_t step, double* __restrict__ zd,
                              double* __restrict__ ze) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    const int64_t nlev = (int64_t)g.nx * g.ny * (g.nz + 1);
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nlev) return;
    const double s2 = 1.4142135623730951;
    const int k = (int)(t / ((int64_t)g.nx * g.ny));
    double a, b;
    if (t < ncell) {
        normal_pair(seed, step, DISCOS_TAG_STRESS_DIAG, 0u, (uint32_t)t, a, b);
        zd[t] = s2 * a;
        zd[t + ncell] = s2 * b;
        normal_pair(seed, step, DISCOS_TAG_STRESS_DIAG, 1u, (uint32_t)t, a, b);
        zd[t + 2 * ncell] = s2 * a;
    }
    normal_pair(seed, step, DISCOS_TAG_STRESS_EDGE, 0u, (uint32_t)t, a, b);
    // wall edges: variance 2 on a no-slip wall, 0 on a slip wall (no tangential stress)
    const double ws = k == 0 ? (g.tsg[0] > 0.0 ? 0.0 : s2)
                             : (k == g.nz ? (g.tsg[1] > 0.0 ? 0.0 : s2) : 1.0);
    ze[t] = ws * a;          // xz
    ze[t + nlev] = ws * b;   // yz
    if (k < g.nz) {
        normal_pair(seed, step, DISCOS_TAG_STRESS_EDGE, 1u, (uint32_t)t, a, b);
        zd[t + 3 * ncell] = a;  // xy
    }
}

// f_out = f_in + amp div_h Z on the faces (the wall faces of w carry f_in unchanged).
__global__ void stress_div_kernel(GridDev g, double amp, const double* __restrict__ zd,
                                  const double* __restrict__ ze, const double* __restrict__ fin,
                                  double* __restrict__ f) {
    const int64_t ncell = (int64_t)g.nx * g.ny * g.nz;
    const int64_t nlev = (int64_t)g.nx * g.ny * (g.nz + 1);
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nlev) return;
    const int nx = g.nx, ny = g.ny;
    const int i = (int)(t % nx), j = (int)((t / nx) % ny), k = (int)(t / ((int64_t)nx * ny));
    const double ih = g.inv_h;
    const int im = (i - 1) & (nx - 1), ip = (i + 1) & (nx - 1);
    const int jm = (j - 1) & (ny - 1), jp = (j + 1) & (ny - 1);
    auto C = [&](int kk, int jj, int ii) { return ((int64_t)kk * ny + jj) * nx + ii; };
    const double* Zxx = zd;
    const double* Zyy = zd + ncell;
    const double* Zzz = zd + 2 * ncell;
    const double* Zxy = zd + 3 * ncell;
    const double* Zxz = ze;
    const double* Zyz = ze + nlev;
    if (k < g.nz) {
        // x-face (i, j+1/2, k+1/2)
        const double fx = (Zxx[C(k, j, i)] - Zxx[C(k, j, im)]) + (Zxy[C(k, jp, i)] - Zxy[C(k, j, i)]) +
                          (Zxz[C(k + 1, j, i)] - Zxz[C(k, j, i)]);
        f[C(k, j, i)] = fin[C(k, j, i)] + amp * ih * fx;
        // y-face (i+1/2, j, k+1/2)
        const double fy = (Zxy[C(k, j, ip)] - Zxy[C(k, j, i)]) + (Zyy[C(k, j, i)] - Zyy[C(k, jm, i)]) +
                          (Zyz[C(k + 1, j, i)] - Zyz[C(k, j, i)]);
        f[ncell + C(k, j, i)] = fin[ncell + C(k, j, i)] + amp * ih * fy;
    }
    if (k >= 1 && k < g.nz) {
        // z-face (i+1/2, j+1/2, k)
        const double fz = (Zxz[C(k, j, ip)] - Zxz[C(k, j, i)]) + (Zyz[C(k, jp, i)] - Zyz[C(k, j, i)]) +
                          (Zzz[C(k, j, i)] - Zzz[C(k - 1, j, i)]);
        f[2 * ncell + C(k, j, i)] = fin[2 * ncell + C(k, j, i)] + amp * ih * fz;
    } else {
        f[2 * ncell + C(k, j, i)] = fin[2 * ncell + C(k, j, i)];
    }
}

// ---- per-mode solve -------------------------------------------------------------

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

// 3x3 real inverse by cofactors.
__device__ __forceinline__ void inv3(const double M[9], double R[9]) {
    const double c00 = M[4] * M[8] - M[5] * M[7];
    const double c01 = M[5] * M[6] - M[3] * M[8];
    const double c02 = M[3] * M[7] - M[4] * M[6];
    const double det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    const double id = 1.0 / det;
    R[0] = c00 * id;
    R[1] = (M[2] * M[7] - M[1] * M[8]) * id;
    R[2] = (M[1] * M[5] - M[2] * M[4]) * id;
    R[3] = c01 * id;
    R[4] = (M[0] * M[8] - M[2] * M[6]) * id;
    R[5] = (M[2] * M[3] - M[0] * M[5]) * id;
    R[6] = c02 * id;
    R[7] = (M[1] * M[6] - M[0] * M[7]) * id;
    R[8] = (M[0] * M[4] - M[1] * M[3]) * id;
}

// The mode systems scaled by 1 / eta (pressure p' = p / eta): eta-free, so their
// factorisation depends only on the grid and is computed once per context.  Per level k
// and mode t, the double2 pairs fac2[(k * SF_P + q) * nmode + t] hold
//   q = 0           (1 / den_k, c'_k) of the scalar tridiagonal (b, or u and v of the
//                   mean flow: -D_zz + kappa^2 with the wall rows of the wall types);
//   q = 1 .. 3      row q-1 of S_k^-1, columns 0 and 1 (S_k the pivot block of (a, w, p);
//                   the continuity row's right-hand side is zero, so column 2 is unused);
//   q = 4 .. 6      row q-4 of C'_k = S_k^-1 C_k, columns 0 and 1 (column 2 of C_k is 0).
// Pairs halve the load instructions per level: the sweeps are bound by the loads a
// wave can keep in flight.
#define SF_P 7

__device__ __forceinline__ void mode_symbols(int t, int nx, int ny, double ih, double2& gx,
                                             double2& gy, double& k2) {
    const int nxh = nx / 2 + 1;
    const int m = t % nxh, n = t / nxh;
    const double tx = 2.0 * M_PI * m / nx, ty = 2.0 * M_PI * n / ny;
    // G = (1 - e^{-i theta}) / h
    gx = make_double2((1.0 - cos(tx)) * ih, sin(tx) * ih);
    gy = make_double2((1.0 - cos(ty)) * ih, sin(ty) * ih);
    k2 = gx.x * gx.x + gx.y * gx.y + gy.x * gy.x + gy.y * gy.y;
}

// Block-Thomas factorisation of every mode (rows E1 a-momentum, E2 w-momentum, E3
// continuity; columns a, w, p; A, B, C the sub-, main and super-diagonal blocks).
__global__ void stokes_factor_kernel(double* __restrict__ fac, int nx, int ny, int nz, double h,
                                     double tsg_lo, double tsg_hi) {
    const int nmode = (nx / 2 + 1) * ny;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nmode) return;
    const size_t st = (size_t)nmode;
    const double ih = 1.0 / h, ih2 = ih * ih;
    double2 gx, gy;
    double k2;
    mode_symbols(t, nx, ny, ih, gx, gy, k2);
    const double kap = sqrt(k2);
    const double off = -ih2;
    const double dgn = 2.0 * ih2 + k2;
    double cb_prev = 0.0;
    double Cprev[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < nz; ++k) {
        double2* f = reinterpret_cast<double2*>(fac) + (size_t)k * SF_P * st + t;
        // ghost u_{-1} = s u_0 of a tangential wall row adds -s / h^2
        const double wall = (k == 0 ? -tsg_lo : 0.0) + (k == nz - 1 ? -tsg_hi : 0.0);
        const double da = dgn + wall * ih2;
        const double den = da - off * cb_prev;
        const double cb = off / den;
        f[0] = make_double2(1.0 / den, cb);
        cb_prev = cb;
        if (t == 0) continue;  // the mean flow uses the scalar factors only (none with two slip walls)
        double B[9] = {da, 0.0, kap, 0.0, dgn, ih, -kap, -ih, 0.0};
        if (k == 0) { B[3] = 0.0; B[4] = 1.0; B[5] = 0.0; }  // w_0 = 0
        if (k > 0) {
            // S = B - A C'_{k-1};  A = [[off,0,0],[0,off,-ih],[0,0,0]]
            B[0] -= off * Cprev[0];
            B[1] -= off * Cprev[1];
            B[2] -= off * Cprev[2];
            B[3] -= off * Cprev[3] - ih * Cprev[6];
            B[4] -= off * Cprev[4] - ih * Cprev[7];
            B[5] -= off * Cprev[5] - ih * Cprev[8];
        }
        double Si[9];
        inv3(B, Si);
        // C = [[off,0,0],[0,off,0],[0,ih,0]] (row 1 of C is 0 at k = 0)
        const double c11 = (k == 0) ? 0.0 : off;
        for (int r = 0; r < 3; ++r) {
            Cprev[3 * r + 0] = Si[3 * r + 0] * off;
            Cprev[3 * r + 1] = Si[3 * r + 1] * c11 + Si[3 * r + 2] * ih;
            Cprev[3 * r + 2] = 0.0;
            f[(1 + r) * st] = make_double2(Si[3 * r + 0], Si[3 * r + 1]);
            f[(4 + r) * st] = make_double2(Cprev[3 * r + 0], Cprev[3 * r + 1]);
        }
    }
}

// Levels a thread's loads run ahead of its sweep: the mode solve has one wave per SIMD
// at most, so the latency of each level's loads is hidden only by loads in flight.
#define SM_AHEAD 8

// Mean flow (kappa = 0): -D_zz u = f / eta with the wall rows for one tangential
// component (col: its [nz] levels at stride st), by the scalar factors of mode 0.
__device__ void mean_flow_component(double2* __restrict__ col, const double2* __restrict__ F,
                                    size_t st, int nz, double sc, double off) {
    double2 br[SM_AHEAD];
    double bf[SM_AHEAD];
#pragma unroll
    for (int j = 0; j < SM_AHEAD; ++j)
        if (j < nz) { br[j] = col[j * st]; bf[j] = F[(size_t)j * SF_P * st].x; }
    double2 d = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < nz; k0 += SM_AHEAD) {
#pragma unroll
        for (int j = 0; j < SM_AHEAD; ++j) {
            const int k = k0 + j;
            if (k < nz) {
                const double2 r = cscale(sc, br[j]);
                const double idn = bf[j];
                if (k + SM_AHEAD < nz) {
                    br[j] = col[(k + SM_AHEAD) * st];
                    bf[j] = F[(size_t)(k + SM_AHEAD) * SF_P * st].x;
                }
                d = cscale(idn, csub(r, cscale(off, d)));
                col[k * st] = d;
            }
        }
    }
    // x_k = d_k - c'_k x_{k+1}, k = nz-2 .. 0 (slot i holds level nz-2-i)
    double2 x = d;
    const int nb = nz - 1;
#pragma unroll
    for (int j = 0; j < SM_AHEAD; ++j)
        if (j < nb) { br[j] = col[(nz - 2 - j) * st]; bf[j] = F[(size_t)(nz - 2 - j) * SF_P * st].y; }
    for (int i0 = 0; i0 < nb; i0 += SM_AHEAD) {
#pragma unroll
        for (int j = 0; j < SM_AHEAD; ++j) {
            const int i = i0 + j;
            if (i < nb) {
                const int k = nz - 2 - i;
                const double2 dk = br[j];
                const double cb = bf[j];
                if (i + SM_AHEAD < nb) {
                    br[j] = col[(k - SM_AHEAD) * st];
                    bf[j] = F[(size_t)(k - SM_AHEAD) * SF_P * st].y;
                }
                x = csub(dk, cscale(cb, x));
                col[k * st] = x;
            }
        }
    }
}

// Mean flow between two slip walls: -D_zz u = f / eta has the constant flow in its
// null space and needs a zero-mean force.  The force's z-mean is removed and the flow
// of zero z-mean taken: with d_{k+1/2} = u_{k+1} - u_k, d_{-1/2} = 0, each row gives
// d_{k+1/2} = -h^2 sum_{j<=k} (g_j - mean g).
__device__ void mean_flow_two_slip(double2* __restrict__ col, size_t st, int nz, double sc, double h2) {
    double2 br[SM_AHEAD];
    double2 fsum = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < SM_AHEAD; ++j)
        if (j < nz) br[j] = col[j * st];
    for (int k0 = 0; k0 < nz; k0 += SM_AHEAD) {
#pragma unroll
        for (int j = 0; j < SM_AHEAD; ++j) {
            const int k = k0 + j;
            if (k < nz) {
                fsum = cadd(fsum, br[j]);
                if (k + SM_AHEAD < nz) br[j] = col[(k + SM_AHEAD) * st];
            }
        }
    }
    const double2 gmean = cscale(sc / nz, fsum);
    double2 G = make_double2(0.0, 0.0), u = G, usum = G;
#pragma unroll
    for (int j = 0; j < SM_AHEAD; ++j)
        if (j < nz) br[j] = col[j * st];
    for (int k0 = 0; k0 < nz; k0 += SM_AHEAD) {
#pragma unroll
        for (int j = 0; j < SM_AHEAD; ++j) {
            const int k = k0 + j;
            if (k < nz) {
                const double2 g = csub(cscale(sc, br[j]), gmean);
                if (k + SM_AHEAD < nz) br[j] = col[(k + SM_AHEAD) * st];
                col[k * st] = u;
                usum = cadd(usum, u);
                G = cadd(G, g);
                u = csub(u, cscale(h2, G));
            }
        }
    }
    const double2 umean = cscale(1.0 / nz, usum);
    for (int k = 0; k < nz; ++k) col[k * st] = csub(col[k * st], umean);
}

// Mean pressure from G_z p = f_z (p_0 = 0, then mean zero) and w = 0.
__device__ void mean_pressure(double2* __restrict__ sw, double2* __restrict__ sp, size_t st, int nz,
                              double hn) {
    double2 bw[SM_AHEAD];
    double2 pk = make_double2(0.0, 0.0), psum = pk;
    for (int pass = 0; pass < 2; ++pass) {
        const double2 mean = cscale(1.0 / nz, psum);
        pk = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < SM_AHEAD; ++j)
            if (j < nz) bw[j] = sw[j * st];
        for (int k0 = 0; k0 < nz; k0 += SM_AHEAD) {
#pragma unroll
            for (int j = 0; j < SM_AHEAD; ++j) {
                const int k = k0 + j;
                if (k < nz) {
                    const double2 wk = bw[j];
                    if (k + SM_AHEAD < nz) bw[j] = sw[(k + SM_AHEAD) * st];
                    if (k > 0) pk = cadd(pk, cscale(hn, wk));
                    if (pass == 0) psum = cadd(psum, pk);
                    else sp[k * st] = csub(pk, mean);
                }
            }
        }
    }
    for (int k = 0; k <= nz; ++k) sw[k * st] = make_double2(0.0, 0.0);
}

// Threads t < nmode: in-plane mode t = n * nxh + m (t = 0: the mean flow's u); t = nmode:
// the mean flow's v; t = nmode + 1: the mean pressure and w.  su, sv, sp: spectra
// [nz][ny][nxh]; sw: [nz+1][ny][nxh].  On entry su, sv, sw hold the force, on exit the
// velocity and sp the pressure.  fac: the factorisation of stokes_factor_kernel.  The
// forward sweep writes y (a, w, p', b) over the inputs, the backward sweep the solution.
__global__ void __launch_bounds__(64)
stokes_mode_kernel(double2* __restrict__ su, double2* __restrict__ sv, double2* __restrict__ sw,
                   double2* __restrict__ sp, const double* __restrict__ fac, int nx, int ny,
                   int nz, double h, double eta, double norm, int two_slip) {
    const int nmode = (nx / 2 + 1) * ny;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nmode + 2) return;
    const size_t st = (size_t)nmode;
    const double ih = 1.0 / h, ih2 = ih * ih;
    const double off = -ih2;
    const double sc = norm / eta;  // scaled right-hand side
    if (t == 0 || t == nmode) {
        if (two_slip) mean_flow_two_slip(t == 0 ? su : sv, st, nz, sc, h * h);
        else mean_flow_component(t == 0 ? su : sv, reinterpret_cast<const double2*>(fac), st, nz, sc, off);
        return;
    }
    if (t == nmode + 1) {
        mean_pressure(sw, sp, st, nz, h * norm);
        return;
    }
    const double2* F = reinterpret_cast<const double2*>(fac) + t;
    double2 gx, gy;
    double k2;
    mode_symbols(t, nx, ny, ih, gx, gy, k2);
    const double ik = 1.0 / sqrt(k2);
    // e = G / kappa; a = e^H u, b = e_perp^H u with e_perp = (-conj gy, conj gx) / kappa
    double2 ya = make_double2(0.0, 0.0), yw = ya, yp = ya, yb = ya;
    {
        double2 bx[SM_AHEAD], by[SM_AHEAD], bz[SM_AHEAD];
        double bf[SM_AHEAD][8];
#pragma unroll
        for (int j = 0; j < SM_AHEAD; ++j) {
            if (j < nz) {
                const size_t o = (size_t)j * st + t;
                bx[j] = su[o];
                by[j] = sv[o];
                bz[j] = j == 0 ? make_double2(0.0, 0.0) : sw[o];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double2 v = F[((size_t)j * SF_P + q) * st];
                    bf[j][2 * q] = v.x;
                    bf[j][2 * q + 1] = v.y;
                }
            }
        }
        for (int k0 = 0; k0 < nz; k0 += SM_AHEAD) {
#pragma unroll
            for (int j = 0; j < SM_AHEAD; ++j) {
                const int k = k0 + j;
                if (k < nz) {
                    const double2 fxk = cscale(sc, bx[j]), fyk = cscale(sc, by[j]), fzk = cscale(sc, bz[j]);
                    double f[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) f[q] = bf[j][q];
                    if (k + SM_AHEAD < nz) {
                        const size_t o = (size_t)(k + SM_AHEAD) * st + t;
                        bx[j] = su[o];
                        by[j] = sv[o];
                        bz[j] = sw[o];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const double2 v = F[((size_t)(k + SM_AHEAD) * SF_P + q) * st];
                            bf[j][2 * q] = v.x;
                            bf[j][2 * q + 1] = v.y;
                        }
                    }
                    const double2 fa = cscale(ik, cadd(cm(cconj(gx), fxk), cm(cconj(gy), fyk)));
                    const double2 fb = cscale(ik, csub(cm(gx, fyk), cm(gy, fxk)));
                    // b: y_b = (f_b - off y_b,prev) / den
                    yb = cscale(f[0], csub(fb, cscale(off, yb)));
                    // (a, w, p'): y = S^-1 (r - A y_prev), r = (f_a, f_z, 0)
                    const double2 r0 = csub(fa, cscale(off, ya));
                    const double2 r1 = csub(fzk, csub(cscale(off, yw), cscale(ih, yp)));
                    ya = cadd(cscale(f[2], r0), cscale(f[3], r1));
                    yw = cadd(cscale(f[4], r0), cscale(f[5], r1));
                    yp = cadd(cscale(f[6], r0), cscale(f[7], r1));
                    const size_t o = (size_t)k * st + t;
                    su[o] = ya;
                    sw[o] = yw;
                    sp[o] = yp;
                    sv[o] = yb;
                }
            }
        }
    }
    // back substitution x_k = y_k - C'_k x_{k+1}; rotate (a, b) back to (u, v)
    double2 xa = ya, xw = yw, xp = yp, xb = yb;
    {
        const size_t o = (size_t)(nz - 1) * st + t;
        su[o] = cscale(ik, csub(cm(xa, gx), cm(xb, cconj(gy))));
        sv[o] = cscale(ik, cadd(cm(xa, gy), cm(xb, cconj(gx))));
        sw[o] = xw;
        sp[o] = cscale(eta, xp);
    }
    const int nb = nz - 1;  // levels nz-2 .. 0; slot j holds level nz-2-i for i = j mod SM_AHEAD
    double2 ba[SM_AHEAD], bw[SM_AHEAD], bp[SM_AHEAD], bb[SM_AHEAD];
    double bc[SM_AHEAD][7];
#pragma unroll
    for (int j = 0; j < SM_AHEAD; ++j) {
        if (j < nb) {
            const int k = nz - 2 - j;
            const size_t o = (size_t)k * st + t;
            ba[j] = su[o]; bw[j] = sw[o]; bp[j] = sp[o]; bb[j] = sv[o];
            bc[j][0] = F[(size_t)k * SF_P * st].y;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double2 v = F[((size_t)k * SF_P + 4 + q) * st];
                bc[j][1 + 2 * q] = v.x;
                bc[j][2 + 2 * q] = v.y;
            }
        }
    }
    for (int i0 = 0; i0 < nb; i0 += SM_AHEAD) {
#pragma unroll
        for (int j = 0; j < SM_AHEAD; ++j) {
            const int i = i0 + j;
            if (i < nb) {
                const int k = nz - 2 - i;
                const double2 y0 = ba[j], y1 = bw[j], y2 = bp[j], y3 = bb[j];
                double c[7];
#pragma unroll
                for (int q = 0; q < 7; ++q) c[q] = bc[j][q];
                if (i + SM_AHEAD < nb) {
                    const int kn = k - SM_AHEAD;
                    const size_t o = (size_t)kn * st + t;
                    ba[j] = su[o]; bw[j] = sw[o]; bp[j] = sp[o]; bb[j] = sv[o];
                    bc[j][0] = F[(size_t)kn * SF_P * st].y;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const double2 v = F[((size_t)kn * SF_P + 4 + q) * st];
                        bc[j][1 + 2 * q] = v.x;
                        bc[j][2 + 2 * q] = v.y;
                    }
                }
                const double2 ta = csub(y0, cadd(cscale(c[1], xa), cscale(c[2], xw)));
                const double2 tw = csub(y1, cadd(cscale(c[3], xa), cscale(c[4], xw)));
                const double2 tp = csub(y2, cadd(cscale(c[5], xa), cscale(c[6], xw)));
                xb = csub(y3, cscale(c[0], xb));
                xa = ta;
                xw = tw;
                xp = tp;
                // u = a e + b e_perp = (a gx - b conj gy) / kappa, v = (a gy + b conj gx) / kappa
                const size_t o = (size_t)k * st + t;
                su[o] = cscale(ik, csub(cm(xa, gx), cm(xb, cconj(gy))));
                sv[o] = cscale(ik, cadd(cm(xa, gy), cm(xb, cconj(gx))));
                sw[o] = (k == 0) ? make_double2(0.0, 0.0) : xw;
                sp[o] = cscale(eta, xp);
            }
        }
    }
    sw[(size_t)nz * st + t] = make_double2(0.0, 0.0);
}

// ---- per-mode solve in segments ----------------------------------------------------
// The same sweeps with SEG_S levels per lane and L = 2^lgL lanes per mode (L SEG_S >= nz,
// L <= 64), so that a mode's levels are worked on in parallel (SEG_S = 4: nz <= 256).  Every sweep is a
// first-order affine recurrence y_k = M_k y_{k-1} + g_k: each lane composes the maps of
// its levels, a Hillis-Steele scan over the lanes (shuffles) composes the prefixes, and
// each lane reruns its levels from the state its predecessors hand it.

__device__ __forceinline__ double2 shfl_up2(double2 v, int d, int w) {
    return make_double2(__shfl_up(v.x, d, w), __shfl_up(v.y, d, w));
}
__device__ __forceinline__ double2 shfl_down2(double2 v, int d, int w) {
    return make_double2(__shfl_down(v.x, d, w), __shfl_down(v.y, d, w));
}
__device__ __forceinline__ double2 shfl_xor2(double2 v, int m, int w) {
    return make_double2(__shfl_xor(v.x, m, w), __shfl_xor(v.y, m, w));
}

// Scalar affine maps y -> a y + b composed over the lanes of a group: on return (a, b)
// is the composition of the maps of lanes 0..lane (forward) or lane..L-1 (backward,
// applied from the top lane down).
template <bool FWD>
__device__ __forceinline__ void scan_affine1(double& a, double2& b, int lane, int L) {
    for (int d = 1; d < L; d <<= 1) {
        const double ap = FWD ? __shfl_up(a, d, L) : __shfl_down(a, d, L);
        const double2 bp = FWD ? shfl_up2(b, d, L) : shfl_down2(b, d, L);
        if (FWD ? lane >= d : lane + d < L) {
            b = cadd(cscale(a, bp), b);
            a = a * ap;
        }
    }
}

// The state handed to this lane: the composed map of the lanes before it applied to 0.
template <bool FWD>
__device__ __forceinline__ double2 handed1(double2 b, int lane, int L) {
    const double2 r = FWD ? shfl_up2(b, 1, L) : shfl_down2(b, 1, L);
    return (FWD ? lane >= 1 : lane + 1 < L) ? r : make_double2(0.0, 0.0);
}

__device__ __forceinline__ double2 group_sum(double2 v, int L) {
    for (int m = 1; m < L; m <<= 1) v = cadd(v, shfl_xor2(v, m, L));
    return v;
}

// 3-vector affine maps Y -> T Y + V (T real 3x3, V complex 3), composed as above.
template <bool FWD>
__device__ __forceinline__ void scan_affine3(double T[9], double2 V[3], int lane, int L) {
    for (int d = 1; d < L; d <<= 1) {
        double Tp[9];
        double2 Vp[3];
#pragma unroll
        for (int q = 0; q < 9; ++q) Tp[q] = FWD ? __shfl_up(T[q], d, L) : __shfl_down(T[q], d, L);
#pragma unroll
        for (int r = 0; r < 3; ++r) Vp[r] = FWD ? shfl_up2(V[r], d, L) : shfl_down2(V[r], d, L);
        if (FWD ? lane >= d : lane + d < L) {
            double2 Vn[3];
            double Tn[9];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                Vn[r] = cadd(V[r], cadd(cadd(cscale(T[3 * r], Vp[0]), cscale(T[3 * r + 1], Vp[1])),
                                        cscale(T[3 * r + 2], Vp[2])));
#pragma unroll
                for (int c2 = 0; c2 < 3; ++c2)
                    Tn[3 * r + c2] = T[3 * r] * Tp[c2] + T[3 * r + 1] * Tp[3 + c2] + T[3 * r + 2] * Tp[6 + c2];
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) T[q] = Tn[q];
#pragma unroll
            for (int r = 0; r < 3; ++r) V[r] = Vn[r];
        }
    }
}

// Mean flow of one tangential component (t = 0) in segments: the tridiagonal sweeps of
// mean_flow_component, or between two slip walls the zero-mean double prefix sum of
// mean_flow_two_slip.
template <int SEG_S>
__device__ void mean_flow_seg(double2* __restrict__ col, const double2* __restrict__ F, size_t st,
                              int nz, double sc, double off, double h2, int two_slip, int lane,
                              int L) {
    double2 g[SEG_S];
    const int k0 = lane * SEG_S;
#pragma unroll
    for (int j = 0; j < SEG_S; ++j)
        g[j] = (k0 + j < nz) ? cscale(sc, col[(k0 + j) * st]) : make_double2(0.0, 0.0);
    if (two_slip) {
        double2 loc = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < SEG_S; ++j) loc = cadd(loc, g[j]);
        const double2 gmean = cscale(1.0 / nz, group_sum(loc, L));
        // G_k = sum_{j<=k} (g_j - mean); u_k = -h^2 sum_{j<k} G_j; then zero mean
        double2 G[SEG_S];
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < SEG_S; ++j) {
            if (k0 + j < nz) acc = cadd(acc, csub(g[j], gmean));
            G[j] = acc;
        }
        double one = 1.0;
        double2 tot = acc;
        scan_affine1<true>(one, tot, lane, L);
        const double2 Gin = handed1<true>(tot, lane, L);
        double2 u[SEG_S];
        double2 uacc = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < SEG_S; ++j) {
            u[j] = uacc;  // exclusive within the lane
            if (k0 + j < nz) uacc = cadd(uacc, cadd(G[j], Gin));
        }
        double one2 = 1.0;
        double2 utot = uacc;
        scan_affine1<true>(one2, utot, lane, L);
        const double2 uin = handed1<true>(utot, lane, L);
        double2 usum = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < SEG_S; ++j) {
            u[j] = cscale(-h2, cadd(u[j], uin));
            if (k0 + j < nz) usum = cadd(usum, u[j]);
        }
        const double2 umean = cscale(1.0 / nz, group_sum(usum, L));
#pragma unroll
        for (int j = 0; j < SEG_S; ++j)
            if (k0 + j < nz) col[(k0 + j) * st] = csub(u[j], umean);
        return;
    }
    // forward: y_k = f0 (g_k - off y_{k-1});  backward: x_k = y_k - c'_k x_{k+1}
    double al[SEG_S], cb[SEG_S];
    double a = 1.0;
    double2 b = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < SEG_S; ++j) {
        const int k = k0 + j;
        if (k < nz) {
            const double2 f = F[(size_t)k * SF_P * st];
            al[j] = -off * f.x;
            g[j] = cscale(f.x, g[j]);
            cb[j] = f.y;
            a = al[j] * a;
            b = cadd(cscale(al[j], b), g[j]);
        } else {
            al[j] = 1.0;
            cb[j] = 0.0;
        }
    }
    scan_affine1<true>(a, b, lane, L);
    double2 y = handed1<true>(b, lane, L);
#pragma unroll
    for (int j = 0; j < SEG_S; ++j) {
        if (k0 + j < nz) {
            y = cadd(cscale(al[j], y), g[j]);
            g[j] = y;
        }
    }
    // backward over the lane's levels from the top; x_{nz-1} = y_{nz-1}
    a = 1.0;
    b = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = SEG_S - 1; j >= 0; --j) {
        const int k = k0 + j;
        if (k < nz) {
            const double m = (k == nz - 1) ? 0.0 : -cb[j];
            cb[j] = m;
            a = m * a;
            b = cadd(cscale(m, b), g[j]);
        }
    }
    scan_affine1<false>(a, b, lane, L);
    double2 x = handed1<false>(b, lane, L);
#pragma unroll
    for (int j = SEG_S - 1; j >= 0; --j) {
        const int k = k0 + j;
        if (k < nz) {
            x = cadd(cscale(cb[j], x), g[j]);
            col[k * st] = x;
        }
    }
}

// Mean pressure in segments (mean_pressure): inclusive prefix sum of h n sw_k (k >= 1),
// zero mean; w = 0.
template <int SEG_S>
__device__ void mean_pressure_seg(double2* __restrict__ sw, double2* __restrict__ sp, size_t st,
                                  int nz, double hn, int lane, int L) {
    const int k0 = lane * SEG_S;
    double2 pk[SEG_S];
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < SEG_S; ++j) {
        const int k = k0 + j;
        if (k >= 1 && k < nz) acc = cadd(acc, cscale(hn, sw[k * st]));
        pk[j] = acc;
    }
    double one = 1.0;
    double2 tot = acc;
    scan_affine1<true>(one, tot, lane, L);
    const double2 pin = handed1<true>(tot, lane, L);
    double2 psum = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < SEG_S; ++j) {
        pk[j] = cadd(pk[j], pin);
        if (k0 + j < nz) psum = cadd(psum, pk[j]);
    }
    const double2 mean = cscale(1.0 / nz, group_sum(psum, L));
#pragma unroll
    for (int j = 0; j < SEG_S; ++j)
        if (k0 + j < nz) sp[(k0 + j) * st] = csub(pk[j], mean);
    for (int k = lane; k <= nz; k += L) sw[k * st] = make_double2(0.0, 0.0);
}

// Groups of L lanes: group t < nmode solves mode t (t = 0: the mean flow's u, v and
// pressure one after the other).  Same inputs and outputs as stokes_mode_kernel.
template <int SEG_S>
__global__ void __launch_bounds__(256)
stokes_mode_seg_kernel(double2* __restrict__ su, double2* __restrict__ sv, double2* __restrict__ sw,
                       double2* __restrict__ sp, const double* __restrict__ fac, int nx, int ny,
                       int nz, double h, double eta, double norm, int two_slip, int lgL) {
    const int nmode = (nx / 2 + 1) * ny;
    const int L = 1 << lgL;
    const int gt = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = gt >> lgL, lane = gt & (L - 1);
    if (t >= nmode) return;  // whole groups: L divides the block
    const size_t st = (size_t)nmode;
    const double ih = 1.0 / h, ih2 = ih * ih;
    const double off = -ih2;
    const double sc = norm / eta;
    const double2* F0 = reinterpret_cast<const double2*>(fac) + t;
    if (t == 0) {
        mean_flow_seg<SEG_S>(su, F0, st, nz, sc, off, h * h, two_slip, lane, L);
        mean_flow_seg<SEG_S>(sv, F0, st, nz, sc, off, h * h, two_slip, lane, L);
        mean_pressure_seg<SEG_S>(sw, sp, st, nz, h * norm, lane, L);
        return;
    }
    double2 gx, gy;
    double k2;
    mode_symbols(t, nx, ny, ih, gx, gy, k2);
    const double ik = 1.0 / sqrt(k2);
    const int k0 = lane * SEG_S;
    // forward maps: Y_k = M_k Y_{k-1} + G_k with M_k = S^-1 [[-off,0,0],[0,-off,ih],[0,0,0]]
    // applied through columns 0, 1 of S^-1; b: yb_k = al_k yb_{k-1} + gb_k
    double si[SEG_S][6];
    double2 G[SEG_S][3], gb[SEG_S];
    double al[SEG_S];
#pragma unroll
    for (int j = 0; j < SEG_S; ++j) {
        const int k = k0 + j;
        if (k < nz) {
            const size_t o = (size_t)k * st + t;
            const double2 fxk = cscale(sc, su[o]), fyk = cscale(sc, sv[o]);
            const double2 fzk = k == 0 ? make_double2(0.0, 0.0) : cscale(sc, sw[o]);
            const double2 f0 = F0[(size_t)k * SF_P * st];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double2 v = F0[((size_t)k * SF_P + 1 + r) * st];
                si[j][2 * r] = v.x;
                si[j][2 * r + 1] = v.y;
            }
            const double2 fa = cscale(ik, cadd(cm(cconj(gx), fxk), cm(cconj(gy), fyk)));
            const double2 fb = cscale(ik, csub(cm(gx, fyk), cm(gy, fxk)));
            al[j] = -off * f0.x;
            gb[j] = cscale(f0.x, fb);
#pragma unroll
            for (int r = 0; r < 3; ++r) G[j][r] = cadd(cscale(si[j][2 * r], fa), cscale(si[j][2 * r + 1], fzk));
        } else {
            al[j] = 1.0;
            gb[j] = make_double2(0.0, 0.0);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                G[j][r] = make_double2(0.0, 0.0);
                si[j][2 * r] = si[j][2 * r + 1] = 0.0;
            }
        }
    }
    auto Mrow = [&](int j, int r, int c2) -> double {  // M_k entries (identity beyond nz)
        if (k0 + j >= nz) return r == c2 ? 1.0 : 0.0;
        return c2 == 0 ? -off * si[j][2 * r] : (c2 == 1 ? -off * si[j][2 * r + 1] : ih * si[j][2 * r + 1]);
    };
    double T[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double2 V[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    double ab = 1.0;
    double2 bb = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < SEG_S; ++j) {
        double Tn[9];
        double2 Vn[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double m0 = Mrow(j, r, 0), m1 = Mrow(j, r, 1), m2 = Mrow(j, r, 2);
            Vn[r] = cadd(G[j][r], cadd(cadd(cscale(m0, V[0]), cscale(m1, V[1])), cscale(m2, V[2])));
#pragma unroll
            for (int c2 = 0; c2 < 3; ++c2) Tn[3 * r + c2] = m0 * T[c2] + m1 * T[3 + c2] + m2 * T[6 + c2];
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) T[q] = Tn[q];
#pragma unroll
        for (int r = 0; r < 3; ++r) V[r] = Vn[r];
        bb = cadd(cscale(al[j], bb), gb[j]);
        ab = al[j] * ab;
    }
    scan_affine3<true>(T, V, lane, L);
    scan_affine1<true>(ab, bb, lane, L);
    double2 y[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) y[r] = handed1<true>(V[r], lane, L);
    double2 yb = handed1<true>(bb, lane, L);
    // rerun: Y_k into G, yb_k into gb
#pragma unroll
    for (int j = 0; j < SEG_S; ++j) {
        if (k0 + j < nz) {
            double2 yn[3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
                yn[r] = cadd(G[j][r], cadd(cadd(cscale(Mrow(j, r, 0), y[0]), cscale(Mrow(j, r, 1), y[1])),
                                           cscale(Mrow(j, r, 2), y[2])));
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                y[r] = yn[r];
                G[j][r] = yn[r];
            }
            yb = cadd(cscale(al[j], yb), gb[j]);
            gb[j] = yb;
        }
    }
    // backward maps: X_k = N_k X_{k+1} + Y_k, N_k = -C'_k (columns 0, 1), N_{nz-1} = 0;
    // xb_k = -c'_k xb_{k+1} + yb_k
    double cn[SEG_S][6];
    double cbm[SEG_S];
#pragma unroll
    for (int j = 0; j < SEG_S; ++j) {
        const int k = k0 + j;
        if (k < nz - 1) {
            cbm[j] = -F0[(size_t)k * SF_P * st].y;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double2 v = F0[((size_t)k * SF_P + 4 + r) * st];
                cn[j][2 * r] = -v.x;
                cn[j][2 * r + 1] = -v.y;
            }
        } else {
            cbm[j] = 0.0;
#pragma unroll
            for (int q = 0; q < 6; ++q) cn[j][q] = 0.0;
        }
    }
    double U[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double2 W[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    ab = 1.0;
    bb = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = SEG_S - 1; j >= 0; --j) {
        if (k0 + j < nz) {
            double Un[9];
            double2 Wn[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double n0 = cn[j][2 * r], n1 = cn[j][2 * r + 1];
                Wn[r] = cadd(G[j][r], cadd(cscale(n0, W[0]), cscale(n1, W[1])));
#pragma unroll
                for (int c2 = 0; c2 < 3; ++c2) Un[3 * r + c2] = n0 * U[c2] + n1 * U[3 + c2];
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) U[q] = Un[q];
#pragma unroll
            for (int r = 0; r < 3; ++r) W[r] = Wn[r];
            bb = cadd(cscale(cbm[j], bb), gb[j]);
            ab = cbm[j] * ab;
        }
    }
    scan_affine3<false>(U, W, lane, L);
    scan_affine1<false>(ab, bb, lane, L);
    double2 x[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) x[r] = handed1<false>(W[r], lane, L);
    double2 xb = handed1<false>(bb, lane, L);
#pragma unroll
    for (int j = SEG_S - 1; j >= 0; --j) {
        const int k = k0 + j;
        if (k < nz) {
            double2 xn[3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
                xn[r] = cadd(G[j][r], cadd(cscale(cn[j][2 * r], x[0]), cscale(cn[j][2 * r + 1], x[1])));
#pragma unroll
            for (int r = 0; r < 3; ++r) x[r] = xn[r];
            xb = cadd(cscale(cbm[j], xb), gb[j]);
            // u = a e + b e_perp = (a gx - b conj gy) / kappa, v = (a gy + b conj gx) / kappa
            const size_t o = (size_t)k * st + t;
            su[o] = cscale(ik, csub(cm(x[0], gx), cm(xb, cconj(gy))));
            sv[o] = cscale(ik, cadd(cm(x[0], gy), cm(xb, cconj(gx))));
            sw[o] = (k == 0) ? make_double2(0.0, 0.0) : x[1];
            sp[o] = cscale(eta, x[2]);
        }
    }
    if (lane == 0) sw[(size_t)nz * st + t] = make_double2(0.0, 0.0);
}

// ---- J^hy -------------------------------------------------------------------------
// V = J^hy v with the wall ghosts: tangential components u_{-1-m} = s u_m (cell
// heights; s = -1 no-slip, +1 slip), normal component w_{-k} = -w_k (faces), mirrored
// at the top.  An ESC window row is read as aligned pairs of doubles (two nodes per
// load; a pair never straddles the x period, nx being even): 5 loads instead of 8 for an
// 8-node row, and as many fewer cache-line lookups in the texture addresser, which
// bounds that gather.  (The 4-point kernel's rows keep their single loads: read as pairs
// they took twice as long, the compiler then batching the window's loads differently.)
__device__ __forceinline__ double face_val(const double* __restrict__ a, const GridDev& g, int comp,
                                           int i, int j, int k) {
    double s = 1.0;
    if (comp < 2) {
        if (k < 0) { k = -1 - k; s = g.tsg[0]; }
        else if (k >= g.nz) { k = 2 * g.nz - 1 - k; s = g.tsg[1]; }
        k = min(max(k, 0), g.nz - 1);
    } else {
        if (k < 0) { k = -k; s = -1.0; }
        else if (k > g.nz) { k = 2 * g.nz - k; s = -1.0; }
        k = min(max(k, 0), g.nz);
    }
    return s * a[((size_t)k * g.ny + j) * g.nx + i];
}

// J^hy v at one position a4 (cell-list ion with kernel row kr when KM != 0): res[3].
// KM = 0: the 4-point Peskin kernel; KM = 2 or 4: the kernel of row kr over a window of
// 2 KM nodes per axis.
template <int KM>
__device__ __forceinline__ void jhy_at(const GridDev& g, const double* __restrict__ vel, double4 a4,
                                       const double* kr, double res[3]) {
    const size_t ncell = (size_t)g.nx * g.ny * g.nz;
    if constexpr (KM != 0) {
        for (int comp = 0; comp < 3; ++comp) {
            const double* a = vel + comp * ncell;
            double wx[2 * KM], wy[2 * KM];
            const int ix0 = hy_axis<KM>(a4.x * g.inv_h - (comp == 0 ? 0.0 : 0.5), kr, wx);
            const int iy0 = hy_axis<KM>(a4.y * g.inv_h - (comp == 1 ? 0.0 : 0.5), kr, wy);
            const double sz = a4.z * g.inv_h - (comp == 2 ? 0.0 : 0.5);
            const int iz0 = (int)floor(sz) + 1 - KM;
            // the row's 2 KM nodes through KM + 1 aligned double pairs (a pair never
            // straddles the period, nx being even): pair k holds nodes e0 + 2k, e0 + 2k + 1
            // with e0 = ix0 rounded down to even; weights shifted by one for an odd ix0
            const bool odd = (ix0 & 1) != 0;
            const int e0 = ix0 - (odd ? 1 : 0);
            double wp[2 * KM + 2];
#pragma unroll
            for (int j = 0; j < 2 * KM + 2; ++j) {
                const double we = j < 2 * KM ? wx[j] : 0.0;
                const double wo = (j >= 1 && j <= 2 * KM) ? wx[j - 1] : 0.0;
                wp[j] = odd ? wo : we;
            }
            int pi[KM + 1];
#pragma unroll
            for (int k = 0; k < KM + 1; ++k) pi[k] = (e0 + 2 * k) & (g.nx - 1);
            double acc = 0.0;
            for (int c = 0; c < 2 * KM; ++c) {
                const double wz = hy_weight(sz - (double)(iz0 + c), kr[0], kr[1], kr[2], kr[3]);
                if (wz == 0.0) continue;
                // no-slip ghost of the level (one fold: nz >= KM)
                int k = iz0 + c;
                double sg = 1.0;
                if (comp < 2) {
                    if (k < 0) { k = -1 - k; sg = g.tsg[0]; }
                    else if (k >= g.nz) { k = 2 * g.nz - 1 - k; sg = g.tsg[1]; }
                    k = min(max(k, 0), g.nz - 1);
                } else {
                    if (k < 0) { k = -k; sg = -1.0; }
                    else if (k > g.nz) { k = 2 * g.nz - k; sg = -1.0; }
                    k = min(max(k, 0), g.nz);
                }
                const double* plane = a + (size_t)k * g.ny * g.nx;
                double accy = 0.0;
#pragma unroll
                for (int b = 0; b < 2 * KM; ++b) {
                    if (wy[b] == 0.0) continue;
                    const double2* rowp = reinterpret_cast<const double2*>(
                        plane + (size_t)((iy0 + b) & (g.ny - 1)) * g.nx);
                    double accx = 0.0;
#pragma unroll
                    for (int k = 0; k < KM + 1; ++k) {
                        const double2 v = rowp[pi[k] >> 1];
                        accx += wp[2 * k] * v.x + wp[2 * k + 1] * v.y;
                    }
                    accy += wy[b] * accx;
                }
                acc += sg * wz * accy;
            }
            res[comp] = acc;
        }
    } else {
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        const double* a = vel + comp * ncell;
        int ix0, iy0, iz0;
        double wx[4], wy[4], wz[4];
        peskin4(a4.x * g.inv_h - (comp == 0 ? 0.0 : 0.5), ix0, wx);
        peskin4(a4.y * g.inv_h - (comp == 1 ? 0.0 : 0.5), iy0, wy);
        peskin4(a4.z * g.inv_h - (comp == 2 ? 0.0 : 0.5), iz0, wz);
        double acc = 0.0;
        for (int c = 0; c < 4; ++c) {
            double accy = 0.0;
            for (int b = 0; b < 4; ++b) {
                const int jj = (iy0 + b) & (g.ny - 1);
                double accx = 0.0;
#pragma unroll
                for (int aa = 0; aa < 4; ++aa)
                    accx += wx[aa] * face_val(a, g, comp, (ix0 + aa) & (g.nx - 1), jj, iz0 + c);
                accy += wy[b] * accx;
            }
            acc += wz[c] * accy;
        }
        res[comp] = acc;
    }
    }
}

// V = J^hy v for the ions xs of the cell list.  midpoint = 0: V at x to out[o]
// (o = perm[i] if scatter) with the given component stride.  midpoint = 1: the two
// stages of eq step1 for the same ion, x* = x + half_dt J(x) v (wrapped in x, y,
// reflected in z) and then J(x*) v to out.  Ion i's kernel: the Peskin kernel (KM = 0) or
// its species' row of the kernel table.
template <int KM>
__global__ void __launch_bounds__(256) interp_hy_kernel(GridDev g, int n, const double4* __restrict__ xs,
                                 const int* __restrict__ perm, const double* __restrict__ vel,
                                 double* __restrict__ out, int64_t stride, int scatter,
                                 int midpoint, double half_dt, int* __restrict__ flags,
                                 const int* __restrict__ ssp, const double* __restrict__ hy_tab) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int o = scatter ? perm[i] : i;
    auto outside = [&](double4 a) {
        set_flag(flags, (isfinite(a.x) && isfinite(a.y) && isfinite(a.z)) ? DISCOS_FLAG_OUT_OF_DOMAIN
                                                                       : DISCOS_FLAG_NONFINITE);
        out[o] = out[o + stride] = out[o + 2 * stride] = 0.0;
    };
    const double4 a4 = xs[i];
    if (!pos_ok(g, a4.x, a4.y, a4.z)) {
        outside(a4);
        return;
    }
    double kr[4] = {0.0, 0.0, 0.0, 0.0};
    if (KM != 0) {
        const double* row = hy_row(hy_tab, ssp[i]);
        kr[0] = row[0]; kr[1] = row[1]; kr[2] = row[2]; kr[3] = row[3];
    }
    double res[3];
    jhy_at<KM>(g, vel, a4, kr, res);
    if (midpoint) {
        const double mx = a4.x + half_dt * res[0], my = a4.y + half_dt * res[1],
                     mz = a4.z + half_dt * res[2];
        double4 m4 = a4;
        if (!(isfinite(mx) && isfinite(my) && isfinite(mz)))
            set_flag(flags, DISCOS_FLAG_NONFINITE);
        else
            m4 = make_double4(wrap_coord(mx, g.Lx), wrap_coord(my, g.Ly), reflect_walls(mz, g.Lz), a4.w);
        if (!pos_ok(g, m4.x, m4.y, m4.z)) {
            outside(m4);
            return;
        }
        jhy_at<KM>(g, vel, m4, kr, res);
    }
    out[o] = res[0];
    out[o + stride] = res[1];
    out[o + 2 * stride] = res[2];
}

template <int KM>
static void interp_hy_launch(Ctx* c, int n, const double* vel, double* out, int64_t stride,
                             int scatter, int midpoint, double half_dt, hipStream_t s) {
    interp_hy_kernel<KM><<<(n + 255) / 256, 256, 0, s>>>(c->gd, n, c->sxyzq, c->perm, vel, out, stride,
                                                        scatter, midpoint, half_dt, c->flags, c->ssp,
                                                        c->hy_tab);
}

static void interp_hy_any(Ctx* c, int species, int n, const double* vel, double* out, int64_t stride,
                          int scatter, int midpoint, double half_dt, hipStream_t s) {
    const int km = species ? c->hy_km : 0;
    if (km == 0) interp_hy_launch<0>(c, n, vel, out, stride, scatter, midpoint, half_dt, s);
    else if (km <= 2) interp_hy_launch<2>(c, n, vel, out, stride, scatter, midpoint, half_dt, s);
    else interp_hy_launch<4>(c, n, vel, out, stride, scatter, midpoint, half_dt, s);
}

int interp_hy_sorted(Ctx* c, int n, const double* vel, double* out, int64_t stride, int scatter,
                     hipStream_t s, int species) {
    if (n <= 0) return DISCOS_OK;
    interp_hy_any(c, species, n, vel, out, stride, scatter, 0, 0.0, s);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

// Stage 4 velocities of the wet step for the ions of the cell list: J(x*) v with the
// predictor x* = x + dt/2 J(x) v, into c->hvi ([3][n_max], sorted); one thread per ion
// takes both gathers.
int midpoint_velocity(Ctx* c, int n, const double* vel, double dt, hipStream_t s, int species) {
    if (n <= 0) return DISCOS_OK;
    interp_hy_any(c, species, n, vel, c->hvi, c->n_max, 0, 1, 0.5 * dt, s);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

// ---- solve ----------------------------------------------------------------------
int fft_rows_r2c(Ctx* c, const double* in, double2* spec, int nrows, hipStream_t s);
int fft_rows_c2r(Ctx* c, const double2* spec, double* out, int nrows, hipStream_t s);
int fft_cols(Ctx* c, double2* spec, int nlev, int inv, hipStream_t s);

// Factorisation of the mode systems of this context's grid (once, at creation).
int stokes_factor(Ctx* c, hipStream_t s) {
    const int nmode = c->gd.nxh * c->gd.ny;
    stokes_factor_kernel<<<(nmode + 63) / 64, 64, 0, s>>>(c->hfac, c->gd.nx, c->gd.ny, c->gd.nz,
                                                         c->grid.h, c->gd.tsg[0], c->gd.tsg[1]);
    c->hfac_key = (c->gd.tsg[0] > 0.0 ? 1 : 0) | (c->gd.tsg[1] > 0.0 ? 2 : 0);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int solve_stokes(Ctx* c, const double* f, const discos_params* p, uint64_t step, int noise,
                 double* vel, double* pres, hipStream_t s) {
    const GridDev& g = c->gd;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t ncell = (size_t)nx * ny * nz;
    const size_t nlev = (size_t)nx * ny * (nz + 1);
    // factors of the current wall types (they are cached per context)
    const int key = (g.tsg[0] > 0.0 ? 1 : 0) | (g.tsg[1] > 0.0 ? 2 : 0);
    if (key != c->hfac_key) {
        const int rcf = stokes_factor(c, s);
        if (rcf) return rcf;
    }
    const double* frhs = f;
    if (noise) {
        // f + amp div Z, built in the velocity buffer (the solve reads it once)
        const double amp = sqrt(2.0 * p->kT * p->eta / (c->grid.h * c->grid.h * c->grid.h * p->dt));
        const int T = 256;
        stress_kernel<<<(int)((nlev + T - 1) / T), T, 0, s>>>(g, p->seed, step, c->hz_diag, c->hz_edge);
        stress_div_kernel<<<(int)((nlev + T - 1) / T), T, 0, s>>>(g, amp, c->hz_diag, c->hz_edge, f, vel);
        frhs = vel;
    }
    const size_t nsp = (size_t)g.nxh * ny;
    double2* su = c->hspec;
    double2* sv = su + nsp * nz;
    double2* sw = sv + nsp * nz;
    double2* sp = sw + nsp * (nz + 1);
    int rc = fft_rows_r2c(c, frhs, su, ny * nz, s);
    if (!rc) rc = fft_rows_r2c(c, frhs + ncell, sv, ny * nz, s);
    if (!rc) rc = fft_rows_r2c(c, frhs + 2 * ncell, sw, ny * (nz + 1), s);
    if (!rc) rc = fft_cols(c, su, nz, 0, s);
    if (!rc) rc = fft_cols(c, sv, nz, 0, s);
    if (!rc) rc = fft_cols(c, sw, nz + 1, 0, s);
    if (rc) return rc;
    const int nmode = g.nxh * ny;
    const double norm = 1.0 / ((double)nx * ny);
    if (nz <= 256) {
        // 4 levels per lane (2 per lane runs slower: the longer scans of 3x3 maps cost
        // more than the occupancy gains); lanes per mode: the power of two covering nz
        int lgL = 0;
        while ((4 << lgL) < nz) ++lgL;
        const int64_t threads = (int64_t)nmode << lgL;
        stokes_mode_seg_kernel<4><<<(int)((threads + 255) / 256), 256, 0, s>>>(
            su, sv, sw, sp, c->hfac, nx, ny, nz, c->grid.h, p->eta, norm, key == 3 ? 1 : 0, lgL);
    } else {
        stokes_mode_kernel<<<(nmode + 2 + 63) / 64, 64, 0, s>>>(su, sv, sw, sp, c->hfac, nx, ny, nz,
                                                           c->grid.h, p->eta, norm, key == 3 ? 1 : 0);
    }
    rc = fft_cols(c, su, nz, 1, s);
    if (!rc) rc = fft_cols(c, sv, nz, 1, s);
    if (!rc) rc = fft_cols(c, sw, nz + 1, 1, s);
    if (!rc && pres) rc = fft_cols(c, sp, nz, 1, s);
    if (!rc) rc = fft_rows_c2r(c, su, vel, ny * nz, s);
    if (!rc) rc = fft_rows_c2r(c, sv, vel + ncell, ny * nz, s);
    if (!rc) rc = fft_rows_c2r(c, sw, vel + 2 * ncell, ny * (nz + 1), s);
    if (!rc && pres) rc = fft_rows_c2r(c, sp, pres, ny * nz, s);
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
