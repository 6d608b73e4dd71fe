// Device-side building blocks shared by the DISCOS kernels (gfx950, FP64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/discos.h"

#define DISCOS_FLAG_OUT_OF_DOMAIN 1
#define DISCOS_FLAG_NOT_NEUTRAL 2
#define DISCOS_FLAG_NONFINITE 4
#define DISCOS_FLAG_BAD_SPECIES 8
#define DISCOS_FLAG_CAPACITY 16  // a tile's candidate rows exceeded its row buffer

// Bin edge of the cell list, in cells: DISCOS_BIN for a single channel (two cells keep the
// near-field search volume small, 5^3 bins for psi = 4 h, and give the spread a one-bin
// halo).  A batch may use 2 or 4 (GridDev::lb); DISCOS_BIN is the smallest edge, which
// the compile-time row bounds of the tile gathers assume.
#define DISCOS_BIN 2
#define DISCOS_LB 1  // log2(DISCOS_BIN)

namespace discos {

struct GridDev {
    int nx, ny, nz, nxh;
    double h, inv_h, Lx, Ly, Lz;
    int nbx, nby, nbz;  // cell-list bins per dimension
    int lb = DISCOS_LB;  // log2 of the bin edge in cells (1: 2 cells, 2: 4 cells)
    // image sign of the tangential velocity components at the lower / upper wall:
    // -1 no-slip, +1 slip (set per hydrodynamic call)
    double tsg[2] = {-1.0, -1.0};
};

// Wall boundary data used by the field kernels.
struct WallDev {
    int type[2];              // DISCOS_BC_*
    const double* value[2];   // [ny][nx] or null (= 0)
    double eps;
    const int* map[2] = {nullptr, nullptr};  // per-column types [ny][nx] (null: type[w])
};

// Type of wall column (i, j) (nx columns per row).
__device__ __forceinline__ int wall_type_at(const WallDev& w, int wall, int i, int j, int nx) {
    return w.map[wall] ? w.map[wall][(size_t)j * nx + i] : w.type[wall];
}

#define DISCOS_FLAG_NOT_CONVERGED 32

// One channel of a batch as the kernels see it: its grid and walls, and where its data
// sit in the batch arrays (cells and spectra grouped by size class, ions and bins in
// channel order).
struct RepDev {
    GridDev g;
    WallDev w;           // wall value pointers already offset to this channel
    int64_t cell_off;    // rho, phi
    int64_t spec_off;    // half spectra and Thomas scratch
    int64_t zg_off;      // z-solve pivots of this channel's grid shape (nz <= 128)
    int bin_off;         // first bin
    int ion_off, n;      // ions [ion_off, ion_off + n)
    double s_lo, s_hi;   // image signs of the two walls
    double scale;        // h^2 / eps / (nx ny), the Poisson right-hand side scale
    int singular;        // both walls Neumann
    int nmode;           // (nx/2 + 1) ny
    uint64_t seed;       // Philox key of this channel's noise
    const double* coef;  // mobility fit [nspecies][2][7]
};

// Workgroups are dispatched to the 8 XCDs round-robin by linear id, and each XCD has its
// own L2.  xcd_block renumbers them (a bijection on [0, nb)) so that XCD x runs one
// contiguous range of logical blocks: gathers whose neighbours sit in nearby blocks
// (cell-list neighbours, tile halos) then find them in the L2 of the XCD that fetched
// them.
#define DISCOS_NXCD 8
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb / DISCOS_NXCD, r = nb % DISCOS_NXCD;
    const int x = b % DISCOS_NXCD, k = b / DISCOS_NXCD;
    return x * q + min(x, r) + k;
}

// (bx, by, bz) of the renumbered block of a 3-D grid.
__device__ __forceinline__ void xcd_block3(int& bx, int& by, int& bz) {
    const int nb = gridDim.x * gridDim.y * gridDim.z;
    const int lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int L = xcd_block(lin, nb);
    bx = L % gridDim.x;
    by = (L / gridDim.x) % gridDim.y;
    bz = L / (gridDim.x * gridDim.y);
}

__device__ __forceinline__ int wrapi(int n, int N) {
    int r = n % N;
    return r < 0 ? r + N : r;
}

__device__ __forceinline__ int floordiv(int a, int b) {
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Positions that the kernels accept: finite, 0 <= z <= Lz, |x|, |y| moderate.
__device__ __forceinline__ bool pos_ok(const GridDev& g, double x, double y, double z) {
    const double big = 1.0e12 * g.h;
    return (z >= 0.0) && (z <= g.Lz) && (fabs(x) < big) && (fabs(y) < big);
}

// 4-point Peskin weights (App. B, eq peskin1d).  For the node set {(n + off) h},
// s = x / h - off, nodes i0 .. i0+3 with i0 = floor(s) - 1 and r = s - floor(s);
// all four branches share q = sqrt(1 + 4 r - 4 r^2):
//   w0 = (3 - 2r - q)/8, w1 = (3 - 2r + q)/8, w2 = (1 + 2r + q)/8, w3 = (1 + 2r - q)/8.
__device__ __forceinline__ void peskin4(double s, int& i0, double w[4]) {
    const double fl = floor(s);
    const double r = s - fl;
    const double q = sqrt(1.0 + 4.0 * r - 4.0 * r * r);
    i0 = (int)fl - 1;
    w[0] = (3.0 - 2.0 * r - q) * 0.125;
    w[1] = (3.0 - 2.0 * r + q) * 0.125;
    w[2] = (1.0 + 2.0 * r + q) * 0.125;
    w[3] = (1.0 + 2.0 * r - q) * 0.125;
}

// x-coordinate in cells, reduced to a bounded range before the int conversion
// (positions may be anywhere on the periodic line).
__device__ __forceinline__ double reduce_periodic(double x, double L) {
    // fmod(x, L) is x on [0, L) and x - L on [L, 2L) exactly (Sterbenz), so the library
    // call is needed only for far excursions
    if (x >= 0.0) {
        if (x < L) return x;
        if (x < 2.0 * L) return x - L;
    } else if (x >= -L) {
        return x + L;
    }
    double r = fmod(x, L);
    return r < 0.0 ? r + L : r;
}

__device__ __forceinline__ void set_flag(int* flags, int f) { atomicOr(flags, f); }

// ---- Philox4x32-10 (Salmon et al., SC'11) ------------------------------------
struct u32x4 {
    uint32_t v[4];
};

__device__ __forceinline__ u32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
        const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    u32x4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

__device__ __forceinline__ double u01(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * 1.1102230246251565e-16;
}

// Two N(0,1) numbers for counter (index, step, tag, pair) and key seed (Box-Muller).
__device__ __forceinline__ void normal_pair(uint64_t seed, uint64_t step, uint32_t tag,
                                            uint32_t pair, uint32_t index, double& n0,
                                            double& n1) {
    u32x4 o = philox4x32_10(index, (uint32_t)(step & 0xFFFFFFFFull), tag, pair,
                            (uint32_t)(seed & 0xFFFFFFFFull), (uint32_t)(seed >> 32));
    const double u1 = u01(o.v[0], o.v[1]);
    const double u2 = u01(o.v[2], o.v[3]);
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 2.0 * M_PI * u2;
    n0 = rad * cos(ang);
    n1 = rad * sin(ang);
}

#define DISCOS_TAG_DRY 1u
#define DISCOS_TAG_STRESS_DIAG 2u
#define DISCOS_TAG_STRESS_EDGE 3u
#define DISCOS_TAG_RFD 4u

// Bin edge of a grid's cell list, in length units.
__host__ __device__ __forceinline__ double bin_edge(const GridDev& g) { return (double)(1 << g.lb) * g.h; }

// Cell-list bin of a position (bins of 2^lb cells; z clamped into the channel).
__device__ __forceinline__ int bin_of(const GridDev& g, double x, double y, double z, int& bx,
                                      int& by, int& bz) {
    int cx = (int)floor(reduce_periodic(x, g.Lx) * g.inv_h);
    int cy = (int)floor(reduce_periodic(y, g.Ly) * g.inv_h);
    int cz = (int)floor(z * g.inv_h);
    cx = min(max(cx, 0), g.nx - 1);
    cy = min(max(cy, 0), g.ny - 1);
    cz = min(max(cz, 0), g.nz - 1);
    bx = cx >> g.lb;
    by = cy >> g.lb;
    bz = cz >> g.lb;
    return (bz * g.nby + by) * g.nbx + bx;
}

// Periodic wrap into [0, L) (-0 and L map to 0).
__device__ __forceinline__ double wrap_coord(double x, double L) {
    double r;
    if (x >= 0.0 && x < 2.0 * L)
        r = x < L ? x : x - L;  // fmod(x, L) exactly
    else if (x < 0.0 && x >= -L)
        r = x;
    else
        r = fmod(x, L);
    if (r < 0.0) r += L;
    if (r >= L) r -= L;
    if (r == 0.0) r = 0.0;
    return r;
}

// Specular reflection at both walls until inside: exact for one crossing, the
// period-2Lz fold of the reflections for anything farther.
__device__ __forceinline__ double reflect_walls(double z, double Lz) {
    if (z >= 0.0 && z <= Lz) return z;
    if (z < 0.0 && z >= -Lz) return -z;
    if (z > Lz && z <= 2.0 * Lz) return 2.0 * Lz - z;
    double t = fmod(z, 2.0 * Lz);
    if (t < 0.0) t += 2.0 * Lz;
    return t <= Lz ? t : 2.0 * Lz - t;
}

// phi at cell (i, j, k), i and j periodic, any k: ghost layer -1-m is 2 phi_b - phi_m
// (Dirichlet) or phi_m + (2m+1) h sigma / eps (Neumann); mirror rule at the top.
__device__ __forceinline__ double phi_at(const double* __restrict__ phi, const GridDev& g,
                                         const WallDev& w, int i, int j, int k) {
    if (k >= 0 && k < g.nz) return phi[((size_t)k * g.ny + j) * g.nx + i];
    const int wall = k < 0 ? 0 : 1;
    const int m = k < 0 ? -1 - k : k - g.nz;
    const int src = min(max(k < 0 ? m : g.nz - 1 - m, 0), g.nz - 1);
    const double base = phi[((size_t)src * g.ny + j) * g.nx + i];
    const double v = w.value[wall] ? w.value[wall][(size_t)j * g.nx + i] : 0.0;
    if (wall_type_at(w, wall, i, j, g.nx) == DISCOS_BC_DIRICHLET) return 2.0 * v - base;
    return base + (2 * m + 1) * g.h * v / w.eps;
}

// Inclusive prefix sum of v over the workgroup (blockDim.x a multiple of 64): shuffles
// within each wavefront, then the wavefront totals through wsum (blockDim.x / 64 ints of
// LDS) after one barrier.  total receives the workgroup's sum.  Before wsum is written
// again the caller needs a barrier.
__device__ __forceinline__ int block_inclusive_scan(int v, int* wsum, int& total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        const int s = wsum[k];
        pre += k < wv ? s : 0;
        tot += s;
    }
    total = tot;
    return x + pre;
}

// Largest number of candidate rows tile_ranges can produce for a tile of ty x tz cells
// starting on even cells (every tile edge is even) with a window of hlo cells below and
// hhi above: each (y, z) bin row of the range contributes at most two x segments.  Bins
// of DISCOS_BIN cells give the most rows; larger bins give fewer.
constexpr int tile_rows_bound(int ty, int tz, int hlo, int hhi) {
    return 2 * ((ty - 1 + hhi) / DISCOS_BIN + (hlo + DISCOS_BIN - 1) / DISCOS_BIN + 1) *
           ((tz - 1 + hhi) / DISCOS_BIN + (hlo + DISCOS_BIN - 1) / DISCOS_BIN + 1);
}

// Cell-list rows of the ions that can reach the nodes of the tile [x0, x0+tx) x
// [y0, y0+ty) x [z0, z0+tz) with a window of hlo cells below and hhi above (cells
// x0-hlo .. x0+tx-1+hhi, periodic in x and y, clipped at the walls in z).  hlo = hhi = 2
// covers the 4-point kernel (a kernel with a window of 2K nodes needs K); kernels shifted
// by up to half a cell (the random finite difference) reach one cell further down.
// Row r gets rstart[r] and the prefix sum rpre[r] of the row lengths (rpre[nr] = total);
// the rows are taken in chunks of blockDim.x, so MAXR may exceed the block (rstart and
// rpre hold MAXR and MAXR + 1 entries, scan blockDim.x).  Returns the row count; the
// caller sizes the tile so that the rows fit in MAXR (tile_rows_bound, checked at
// compile time by each caller).  Rows beyond MAXR would be dropped: that sets the
// sticky DISCOS_FLAG_CAPACITY in flags, so the loss cannot go unreported.
template <int MAXR>
__device__ int tile_ranges(const GridDev& g, const int* __restrict__ bin_start, int x0, int y0,
                             int z0, int tx, int ty, int tz, int* rstart, int* rpre, int* scan,
                             int* __restrict__ flags, int hlo = 2, int hhi = 2) {
    int sa[2], sb[2], nseg;
    {
        // arithmetic shifts: floor division by the bin edge, negative cells included
        const int lo = (x0 - hlo) >> g.lb, hi = (x0 + tx - 1 + hhi) >> g.lb;
        if (hi - lo + 1 >= g.nbx) {
            nseg = 1; sa[0] = 0; sb[0] = g.nbx - 1;
        } else {
            const int a = wrapi(lo, g.nbx), b = wrapi(hi, g.nbx);
            if (a <= b) { nseg = 1; sa[0] = a; sb[0] = b; }
            else { nseg = 2; sa[0] = a; sb[0] = g.nbx - 1; sa[1] = 0; sb[1] = b; }
        }
    }
    int ylo = (y0 - hlo) >> g.lb, yhi = (y0 + ty - 1 + hhi) >> g.lb;
    if (yhi - ylo + 1 >= g.nby) { ylo = 0; yhi = g.nby - 1; }
    const int czlo = max(z0 - hlo, 0), czhi = min(z0 + tz - 1 + hhi, g.nz - 1);
    const int bzlo = czlo >> g.lb, bzhi = czhi >> g.lb;
    const int nyb = yhi - ylo + 1;
    const int ncand = max(bzhi - bzlo + 1, 0) * nyb * nseg;
    const int t = threadIdx.x, bd = blockDim.x;
    if (ncand > MAXR && t == 0) set_flag(flags, DISCOS_FLAG_CAPACITY);
    const int nr = max(min(ncand, MAXR), 1);
    int carry = 0;
    for (int base = 0; base < nr; base += bd) {
        const int r = base + t;
        int len = 0;
        if (r < ncand && r < MAXR) {
            const int sgi = r % nseg;
            const int yy = ylo + (r / nseg) % nyb;
            const int bz = bzlo + r / (nseg * nyb);
            const int row = (bz * g.nby + wrapi(yy, g.nby)) * g.nbx;
            const int st = bin_start[row + sa[sgi]];
            rstart[r] = st;
            len = bin_start[row + sb[sgi] + 1] - st;
        }
        int tot;
        const int inc = block_inclusive_scan(len, scan, tot);
        if (r < nr) rpre[r] = carry + inc - len;
        carry += tot;
        __syncthreads();  // scan (the wavefront totals) is rewritten by the next chunk
    }
    if (t == 0) {
        rpre[nr] = (ncand > 0) ? carry : 0;
        if (ncand == 0) { rstart[0] = 0; rpre[0] = 0; }
    }
    __syncthreads();
    return nr;
}

}  // namespace discos
