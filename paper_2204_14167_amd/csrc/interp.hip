// J^es: interpolation of the electric field E = -grad_h phi to the ions (eq efieldop,
// eq kernel1) with ghost values beyond the walls filled from the wall conditions
// (Sec. II.B.1: ghosts satisfy the boundary condition on phi).
//
// E lives on the faces of the cell-centred phi (the staggered location of grad_h).
// For an ion in cell (cx, cy, cz) every node any component needs lies in the 5^3
// window of cells cx-2 .. cx+2 (likewise y, z), so the face differences fold into
// per-dimension "derivative weights" and the three components become
//   E_x = -(1/h) sum_z wc_z sum_y wc_y sum_x dw_x phi,
//   E_y = -(1/h) sum_z wc_z sum_y dw_y sum_x wc_x phi,
//   E_z = -(1/h) sum_z dw_z sum_y wc_y sum_x wc_x phi,
// with wc the centre-node Peskin weights and dw_k = wf_{k-1} - wf_k the differences of
// the face-node weights: 125 loads per ion instead of 240.
//
// One workgroup owns a tile of cells, stages phi on the tile plus its halo in LDS
// (ghost layers included, so the gathers have no branches), and interpolates every
// ion of the tile from the cell list.  Tiles without ions stage nothing; tiles with a
// few ions (sparse channels of a batch) read their windows straight from memory.
#include "kernels.h"

namespace discos {

#define IT_TX 16
#define IT_TY 16
#define IT_TZ 8
#define IT_H 5  // halo cells: 2 below, 3 above (an ion exactly on x = L or z = Lz)
#define IT_THREADS 256
#define IT_MAXR 64

// Centre weights and face-difference weights on the 5-cell window c-2 .. c+2 of the
// coordinate u (in cells).
__device__ __forceinline__ int window_weights(double u, double wc5[5], double dw5[5]) {
    int ic, iff;
    double wc[4], wf[4];
    peskin4(u - 0.5, ic, wc);
    peskin4(u, iff, wf);
    const int c = iff + 1;  // floor(u)
    const bool shift = (ic - (c - 2)) != 0;  // centre window starts at c-2 or c-1
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double lo = (k < 4) ? wc[k] : 0.0;
        const double hi = (k > 0) ? wc[k - 1] : 0.0;
        wc5[k] = shift ? hi : lo;
    }
    // faces c-1 .. c+2 use cells (c-2, c-1) .. (c+1, c+2)
    dw5[0] = -wf[0];
    dw5[1] = wf[0] - wf[1];
    dw5[2] = wf[1] - wf[2];
    dw5[3] = wf[2] - wf[3];
    dw5[4] = wf[3];
    return c;
}

// Weighted sums over the 5^3 window whose first node is (lx0, ly0, lz0) of the array
// that fetch(x, y, z) reads: returns E_x, E_y, E_z times -h and the potential P.  UY
// unrolls the y loop (the loads of UY rows in flight at once).
template <int UY, class F>
__device__ __forceinline__ void window_sums(const F& fetch, const double wcx[5], const double dwx[5],
                                            const double wcy[5], const double dwy[5],
                                            const double wcz[5], const double dwz[5], double& Ex,
                                            double& Ey, double& Ez, double& P) {
    Ex = Ey = Ez = P = 0.0;
#pragma unroll 1
    for (int kz = 0; kz < 5; ++kz) {
        double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll UY
        for (int ky = 0; ky < 5; ++ky) {
            double d = 0.0, c = 0.0;
#pragma unroll
            for (int kx = 0; kx < 5; ++kx) {
                const double v = fetch(kx, ky, kz);
                d += dwx[kx] * v;
                c += wcx[kx] * v;
            }
            ax += wcy[ky] * d;
            ay += dwy[ky] * c;
            az += wcy[ky] * c;
        }
        Ex += wcz[kz] * ax;
        Ey += wcz[kz] * ay;
        Ez += dwz[kz] * az;
        P += wcz[kz] * az;
    }
}

// Tiles with at most this many ions gather phi straight from memory (125 loads per ion)
// instead of staging the (TX+5)(TY+5)(TZ+5) window: sparse channels of a batch.
#define IT_DIRECT 16
// Staging loads in flight per thread.
#define IT_UNROLL 8

// One tile of TX x TY x TZ cells (clipped to the grid) starting at (x0, y0, z0):
// find the tile's ions in the cell list; if there are any, stage phi with its halo and
// ghost layers in LDS (tile holds (TX+5)(TY+5)(TZ+5) doubles) or, for a few ions, read
// it directly, and interpolate every ion of the tile's cells.
// The window sums of an ion in cell (cx, cy, cz) read straight from phi (no staged
// tile): ghost rules only where the window reaches past a wall.
__device__ __forceinline__ void direct_sums(const GridDev& g, const WallDev& w,
                                            const double* __restrict__ phi, int cx, int cy, int cz,
                                            const double wcx[5], const double dwx[5],
                                            const double wcy[5], const double dwy[5],
                                            const double wcz[5], const double dwz[5], double& Ex,
                                            double& Ey, double& Ez, double& P) {
    const int nx1 = g.nx - 1, ny1 = g.ny - 1;
    if (cz >= 2 && cz + 2 < g.nz) {
        // window cells cx-2 .. cx+2 (likewise y, z), all inside the channel
        window_sums<1>(
            [&](int kx, int ky, int kz) {
                return phi[((size_t)(cz - 2 + kz) * g.ny + ((cy - 2 + ky) & ny1)) * g.nx +
                           ((cx - 2 + kx) & nx1)];
            },
            wcx, dwx, wcy, dwy, wcz, dwz, Ex, Ey, Ez, P);
    } else {
        window_sums<1>(
            [&](int kx, int ky, int kz) {
                return phi_at(phi, g, w, (cx - 2 + kx) & nx1, (cy - 2 + ky) & ny1, cz - 2 + kz);
            },
            wcx, dwx, wcy, dwy, wcz, dwz, Ex, Ey, Ez, P);
    }
}

template <int TX, int TY, int TZ, bool EARLY = false>
__device__ __forceinline__ void interp_tile(const GridDev& g, const WallDev& w, int op,
                                            const double4* __restrict__ sxyzq,
                                            const int* __restrict__ bin_start,
                                            const int* __restrict__ perm,
                                            const double* __restrict__ phi, double ex0, double ex1,
                                            double ex2, double* __restrict__ out, int64_t stride,
                                            int scatter, int* __restrict__ flags, int x0, int y0,
                                            int z0, double* tile, int* rstart, int* rpre, int* scan) {
    constexpr int LX = TX + IT_H, LY = TY + IT_H;
    const int tx = min(TX, g.nx), ty = min(TY, g.ny);
    const int tz = min(TZ, g.nz - z0);
    const int lxn = tx + IT_H, lyn = ty + IT_H, lzn = tz + IT_H;
    // ions of the tile: rows (bz, by) of tx / 2^lb contiguous bins (tile edges fall on bin edges)
    const int nbxt = tx >> g.lb, nbyt = ty >> g.lb;
    const int bz0 = z0 >> g.lb, bz1 = (z0 + tz - 1) >> g.lb;
    const int nrows = (bz1 - bz0 + 1) * nbyt;
    constexpr int PLANE = LX * LY;
    const bool inner = z0 >= 2 && z0 + tz + 3 <= g.nz;  // no ghost layer in the window
    const size_t pstride = (size_t)g.nx * g.ny;
    // EARLY (a single channel, where nearly every tile holds ions): an inner tile's phi
    // window is loaded into registers before the row scan, so that its loads and the
    // bin-start loads are in flight together; the values go to LDS after the scan (an
    // empty tile has then read its window for nothing)
    constexpr int NCOL = (PLANE + IT_THREADS - 1) / IT_THREADS, LZW = TZ + IT_H;
    double early[EARLY ? NCOL : 1][EARLY ? LZW : 1];
    if (EARLY && inner) {
#pragma unroll
        for (int k = 0; k < NCOL; ++k) {
            const int pp = threadIdx.x + k * IT_THREADS;
            const int lx = pp % LX, ly = pp / LX;
            const bool in = pp < PLANE && lx < lxn && ly < lyn;
            const int i = (x0 - 2 + lx) & (g.nx - 1), j = (y0 - 2 + ly) & (g.ny - 1);
            const double* src = phi + (size_t)(z0 - 2) * pstride + (size_t)j * g.nx + i;
#pragma unroll
            for (int u = 0; u < LZW; ++u)
                early[k][u] = (in && u < lzn) ? src[(size_t)u * pstride] : 0.0;
        }
    }
    {
        // thread t < nrows owns row t; a workgroup scan of the row lengths gives rpre
        int len = 0;
        const int t = threadIdx.x;
        if (t < nrows) {
            const int bz = bz0 + t / nbyt, by = (y0 >> g.lb) + t % nbyt;
            const int row = (bz * g.nby + by) * g.nbx + (x0 >> g.lb);
            const int st = bin_start[row];
            rstart[t] = st;
            len = bin_start[row + nbxt] - st;
        }
        int tot;
        const int inc = block_inclusive_scan(len, scan, tot);
        if (t < nrows) rpre[t] = inc - len;
        if (t == nrows - 1) rpre[nrows] = inc;
    }
    __syncthreads();
    const int total = rpre[nrows];
    if (total == 0) return;  // the same for the whole workgroup
    const bool direct = total <= IT_DIRECT;
    if (EARLY && inner) {
#pragma unroll
        for (int k = 0; k < NCOL; ++k) {
            const int pp = threadIdx.x + k * IT_THREADS;
            if (pp < PLANE) {
#pragma unroll
                for (int u = 0; u < LZW; ++u)
                    if (u < lzn) tile[u * PLANE + pp] = early[k][u];
            }
        }
        __syncthreads();
    } else if (!direct) {
        // phi on cells [x0-2, x0+tx+3) x [y0-2, y0+ty+3) x [z0-2, z0+tz+3), ghosts filled:
        // each thread takes whole z columns of the window (no index divisions per element),
        // with IT_UNROLL loads in flight before the LDS stores
        for (int pp = threadIdx.x; pp < PLANE; pp += IT_THREADS) {
            const int lx = pp % LX, ly = pp / LX;
            const bool in_xy = lx < lxn && ly < lyn;
            const int i = (x0 - 2 + lx) & (g.nx - 1), j = (y0 - 2 + ly) & (g.ny - 1);
            if (inner) {
                const double* src = phi + (size_t)(z0 - 2) * pstride + (size_t)j * g.nx + i;
                for (int lz0 = 0; lz0 < lzn; lz0 += IT_UNROLL) {
                    double v[IT_UNROLL];
#pragma unroll
                    for (int u = 0; u < IT_UNROLL; ++u)
                        v[u] = (lz0 + u < lzn && in_xy) ? src[(size_t)(lz0 + u) * pstride] : 0.0;
#pragma unroll
                    for (int u = 0; u < IT_UNROLL; ++u)
                        if (lz0 + u < lzn) tile[(lz0 + u) * PLANE + pp] = v[u];
                }
            } else {
                for (int lz = 0; lz < lzn; ++lz)
                    tile[lz * PLANE + pp] = in_xy ? phi_at(phi, g, w, i, j, z0 - 2 + lz) : 0.0;
            }
        }
        __syncthreads();
    }
    for (int f = threadIdx.x; f < total; f += blockDim.x) {
        int r = 0, hi = nrows - 1;
        while (r < hi) {  // last row with rpre[row] <= f
            const int mid = (r + hi + 1) >> 1;
            if (rpre[mid] <= f)
                r = mid;
            else
                hi = mid - 1;
        }
        const int i = rstart[r] + (f - rpre[r]);
        const int o = scatter ? perm[i] : i;
        const double4 a4 = sxyzq[i];
        bool ok = pos_ok(g, a4.x, a4.y, a4.z);
        double wcx[5], dwx[5], wcy[5], dwy[5], wcz[5], dwz[5];
        int cx = 0, cy = 0, cz = 0, lx0 = 0, ly0 = 0, lz0 = 0;
        if (ok) {
            cx = window_weights(a4.x * g.inv_h, wcx, dwx);
            cy = window_weights(a4.y * g.inv_h, wcy, dwy);
            cz = window_weights(a4.z * g.inv_h, wcz, dwz);
            lx0 = (cx - x0) & (g.nx - 1);
            ly0 = (cy - y0) & (g.ny - 1);
            lz0 = cz - z0;
            ok = lx0 >= 0 && lx0 <= tx && ly0 >= 0 && ly0 <= ty && lz0 >= 0 && lz0 <= tz;
        }
        if (!ok) {
            set_flag(flags, (isfinite(a4.x) && isfinite(a4.y) && isfinite(a4.z))
                                ? DISCOS_FLAG_OUT_OF_DOMAIN
                                : DISCOS_FLAG_NONFINITE);
            out[o] = 0.0;
            if (op != DISCOS_INTERP_PHI) {
                out[o + stride] = 0.0;
                out[o + 2 * stride] = 0.0;
            }
            continue;
        }
        double Ex, Ey, Ez, P;
        if (!direct) {
            const double* base = &tile[(lz0 * LY + ly0) * LX + lx0];
            window_sums<5>([&](int kx, int ky, int kz) { return base[(kz * LY + ky) * LX + kx]; },
                        wcx, dwx, wcy, dwy, wcz, dwz, Ex, Ey, Ez, P);
        } else {
            direct_sums(g, w, phi, cx, cy, cz, wcx, dwx, wcy, dwy, wcz, dwz, Ex, Ey, Ez, P);
        }
        if (op == DISCOS_INTERP_PHI) {
            out[o] = P;
            continue;
        }
        Ex *= -g.inv_h;
        Ey *= -g.inv_h;
        Ez *= -g.inv_h;
        if (op == DISCOS_INTERP_FORCE) {
            const double qi = a4.w;
            Ex = qi * (Ex + ex0);
            Ey = qi * (Ey + ex1);
            Ez = qi * (Ez + ex2);
        }
        out[o] = Ex;
        out[o + stride] = Ey;
        out[o + 2 * stride] = Ez;
    }
}

__global__ void __launch_bounds__(IT_THREADS)
interp_es_kernel(GridDev g, WallDev w, int op, const double4* __restrict__ sxyzq,
                 const int* __restrict__ bin_start, const int* __restrict__ perm,
                 const double* __restrict__ phi, double ex0, double ex1, double ex2,
                 double* __restrict__ out, int64_t stride, int scatter, int* __restrict__ flags) {
    __shared__ double tile[(IT_TZ + IT_H) * (IT_TY + IT_H) * (IT_TX + IT_H)];
    __shared__ int rstart[IT_MAXR], rpre[IT_MAXR + 1], scan[IT_THREADS];
    const int tx = min(IT_TX, g.nx), ty = min(IT_TY, g.ny);
    int bx, by, bz;
    xcd_block3(bx, by, bz);
    interp_tile<IT_TX, IT_TY, IT_TZ, true>(g, w, op, sxyzq, bin_start, perm, phi, ex0, ex1, ex2,
                                           out, stride, scatter, flags, bx * tx, by * ty, bz * IT_TZ,
                                           tile, rstart, rpre, scan);
}

// Batched: forces q (E^P + E_ext) of every channel's ions, in cell-list order; the
// persistent grid walks the (channel, tile) tasks.
template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(IT_THREADS)
interp_es_batch_kernel(const RepDev* __restrict__ reps, const int2* __restrict__ tasks,
                       int ntasks, const double4* __restrict__ sxyzq,
                       const int* __restrict__ bin_start, const int* __restrict__ perm,
                       const double* __restrict__ phi, double ex0, double ex1, double ex2,
                       double* __restrict__ out, int64_t stride, const int* __restrict__ idirect,
                       int* __restrict__ flags) {
    __shared__ double tile[(TZ + IT_H) * (TY + IT_H) * (TX + IT_H)];
    __shared__ int rstart[IT_MAXR], rpre[IT_MAXR + 1], scan[IT_THREADS];
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const int2 task = tasks[t];
        if (idirect[task.x]) continue;  // interpolated one thread per ion
        const RepDev& R = reps[task.x];
        const GridDev g = R.g;
        const int tx = min(TX, g.nx), ty = min(TY, g.ny);
        const int ntx = g.nx / tx, nty = g.ny / ty;
        const int k = task.y;
        interp_tile<TX, TY, TZ>(g, R.w, DISCOS_INTERP_FORCE, sxyzq, bin_start + R.bin_off, perm,
                                phi + R.cell_off, ex0, ex1, ex2, out, stride, 0, flags,
                                (k % ntx) * tx, ((k / ntx) % nty) * ty, (k / (ntx * nty)) * TZ,
                                tile, rstart, rpre, scan);
        __syncthreads();
    }
}

// Batched, the channels flagged in idirect (few ions per tile, where staging a tile
// would serve a handful of ions): one thread per ion, its window read from phi.
__global__ void __launch_bounds__(256)
interp_es_direct_batch_kernel(const RepDev* __restrict__ reps, const int* __restrict__ ion_rep,
                              const int* __restrict__ idirect, int n, const double4* __restrict__ sxyzq,
                              const double* __restrict__ phi, double ex0, double ex1, double ex2,
                              double* __restrict__ out, int64_t stride, int* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = ion_rep[i];
    if (!idirect[r]) return;
    const RepDev& R = reps[r];
    const GridDev& g = R.g;
    const double4 a4 = sxyzq[i];
    if (!pos_ok(g, a4.x, a4.y, a4.z)) {
        set_flag(flags, (isfinite(a4.x) && isfinite(a4.y) && isfinite(a4.z)) ? DISCOS_FLAG_OUT_OF_DOMAIN
                                                                          : DISCOS_FLAG_NONFINITE);
        out[i] = out[i + stride] = out[i + 2 * stride] = 0.0;
        return;
    }
    double wcx[5], dwx[5], wcy[5], dwy[5], wcz[5], dwz[5];
    const int cx = window_weights(a4.x * g.inv_h, wcx, dwx);
    const int cy = window_weights(a4.y * g.inv_h, wcy, dwy);
    const int cz = window_weights(a4.z * g.inv_h, wcz, dwz);
    double Ex, Ey, Ez, P;
    direct_sums(g, R.w, phi + R.cell_off, cx, cy, cz, wcx, dwx, wcy, dwy, wcz, dwz, Ex, Ey, Ez, P);
    const double qi = a4.w;
    out[i] = qi * (-g.inv_h * Ex + ex0);
    out[i + stride] = qi * (-g.inv_h * Ey + ex1);
    out[i + 2 * stride] = qi * (-g.inv_h * Ez + ex2);
}

int interp_es_sorted(Ctx* c, int op, int n, const double* phi, const discos_params* p,
                     double* out, int64_t out_stride, int scatter, hipStream_t s) {
    if (n <= 0) return DISCOS_OK;
    const GridDev& g = c->gd;
    const int tx = std::min(IT_TX, g.nx), ty = std::min(IT_TY, g.ny);
    dim3 grid(g.nx / tx, g.ny / ty, (g.nz + IT_TZ - 1) / IT_TZ);
    interp_es_kernel<<<grid, IT_THREADS, 0, s>>>(g, wall_of(p), op, c->sxyzq, c->bin_start, c->perm,
                                                 phi, p->e_ext[0], p->e_ext[1], p->e_ext[2], out,
                                                 out_stride, scatter, c->flags);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int batch_interp(Batch* b, hipStream_t s) {
    const int v = b->cfg.interp_t == 8 ? 0 : 1;
    const int nt = b->ntasks[1][v];
    if (nt == 0) return DISCOS_OK;
    const int nb = b->cfg.interp_blocks > 0 ? std::min(nt, b->cfg.interp_blocks) : nt;
    const double* e = b->p.e_ext;
    if (b->n_direct == (int)b->reps.size()) {
        // every channel one thread per ion: no tiles
    } else if (v == 0)
        interp_es_batch_kernel<8, 8, 8><<<nb, IT_THREADS, 0, s>>>(
            b->reps_d, b->tasks[1][0], nt, b->sxyzq, b->bin_start, b->perm, b->phi, e[0], e[1], e[2],
            b->fp, b->n_tot, b->idirect, b->flags);
    else
        interp_es_batch_kernel<IT_TX, IT_TY, IT_TZ><<<nb, IT_THREADS, 0, s>>>(
            b->reps_d, b->tasks[1][1], nt, b->sxyzq, b->bin_start, b->perm, b->phi, e[0], e[1], e[2],
            b->fp, b->n_tot, b->idirect, b->flags);
    if (b->n_direct > 0)
        interp_es_direct_batch_kernel<<<(int)((b->n_tot + 255) / 256), 256, 0, s>>>(
            b->reps_d, b->ion_rep, b->idirect, (int)b->n_tot, b->sxyzq, b->phi, e[0], e[1], e[2], b->fp,
            b->n_tot, b->flags);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
