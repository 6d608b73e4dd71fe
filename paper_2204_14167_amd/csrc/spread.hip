// S^es: charge spreading with the 4-point Peskin kernel and image folding at the
// walls (eq kernel2, Sec. II.A image construction, Sec. II.B.1 image signs).
//
// One workgroup owns a tile of cells and accumulates into LDS every contribution
// that lands in it: it gathers the ions of the tile and of a two-cell halo from the
// cell list (one bin of DISCOS_BIN cells), computes each ion's weights once, adds
// the products that fall inside the tile with LDS atomics, and writes the tile to
// HBM once with coalesced stores.  No global atomics and no zero-fill of the output.
#include "kernels.h"

namespace discos {

// A single channel's tiles: 16 x 16 x 32 cells (64 KB of LDS) with 512 threads; the tiles
// of a batch: 8^3 or 16^3 with 256 threads.
#define SP_TX 16
#define SP_TY 16
#define SP_TZ 32
#define SP_THREADS_ONE 512
#define SP_MAXR_ONE 512
#define SP_THREADS 256
#define SP_MAXR 256


__device__ __forceinline__ int find_range(const int* rpre, int nr, int f) {
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rpre[mid] <= f)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One tile [x0, x0 + T) x [y0, y0 + T) x [z0, z0 + TZ) (clipped to the grid): gather the
// ions of the tile and its halo, accumulate in LDS, store once.  acc holds T^2 TZ doubles.
// MIXED: a wall may have a per-column type map, whose fold sign is then looked up per
// node; with uniform walls (MIXED = false) the fold sign is one factor per layer.
template <int T, bool MIXED = false, int TZ = T, int MAXR = SP_MAXR>
__device__ __forceinline__ void spread_tile(const GridDev& g, const double4* __restrict__ sxyzq,
                                            const int* __restrict__ bin_start, double sign_lo,
                                            double sign_hi, int add_bc, const WallDev& wall,
                                            double* __restrict__ out, int x0, int y0, int z0,
                                            double* acc, int* rstart, int* rpre, int* scan,
                                            int* __restrict__ flags, bool gather = true) {
    static_assert(tile_rows_bound(T, TZ, 2, 2) <= MAXR, "spread tile rows exceed MAXR");
    const int tx = min(T, g.nx), ty = min(T, g.ny);
    const int tz = min(TZ, g.nz - z0);
    const int ncell = tx * ty * tz;
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) acc[k] = 0.0;
    int nr = 1, total = 0;
    if (gather) {  // else the tile stores its wall terms only (ions added by the caller)
        nr = tile_ranges<MAXR>(g, bin_start, x0, y0, z0, tx, ty, tz, rstart, rpre, scan, flags);
        total = rpre[nr];
    } else {
        __syncthreads();  // acc cleared
    }
    const double inv_h3 = g.inv_h * g.inv_h * g.inv_h;
    // the next ion's record is loaded before the current one's LDS atomics
    double4 nxt = make_double4(0.0, 0.0, 0.0, 0.0);
    if ((int)threadIdx.x < total) {
        const int r = find_range(rpre, nr, threadIdx.x);
        nxt = sxyzq[rstart[r] + ((int)threadIdx.x - rpre[r])];
    }
    for (int f = threadIdx.x; f < total; f += blockDim.x) {
        const double4 a4 = nxt;
        const int fn = f + blockDim.x;
        if (fn < total) {
            const int r = find_range(rpre, nr, fn);
            nxt = sxyzq[rstart[r] + (fn - rpre[r])];
        }
        const double x = a4.x, y = a4.y, z = a4.z;
        if (!pos_ok(g, x, y, z)) continue;
        int ix0, iy0, iz0;
        double wx[4], wy[4], wz[4];
        // x, y of the cell list are already reduced into [0, L]
        peskin4(x * g.inv_h - 0.5, ix0, wx);
        peskin4(y * g.inv_h - 0.5, iy0, wy);
        peskin4(z * g.inv_h - 0.5, iz0, wz);
        const double scale = a4.w * inv_h3;
        int lxs[4], lys[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) lxs[a] = (ix0 + a - x0) & (g.nx - 1);
#pragma unroll
        for (int b = 0; b < 4; ++b) lys[b] = (iy0 + b - y0) & (g.ny - 1);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            int kz = iz0 + c;
            double sgn = 1.0;
            const int* fmap = nullptr;  // folded onto a wall of mixed type: sign per column
            if (kz < 0) {
                kz = -1 - kz;
                sgn = sign_lo;
                if (MIXED) fmap = wall.map[0];
            } else if (kz >= g.nz) {
                kz = 2 * g.nz - 1 - kz;
                sgn = sign_hi;
                if (MIXED) fmap = wall.map[1];
            }
            const int lz = kz - z0;
            if (lz < 0 || lz >= tz) continue;
            const double wzc = scale * (fmap ? 1.0 : sgn) * wz[c];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (lys[b] >= ty) continue;
                const double wyz = wzc * wy[b];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    if (lxs[a] >= tx) continue;
                    double v = wyz * wx[a];
                    if (MIXED && fmap &&
                        fmap[(size_t)((iy0 + b) & (g.ny - 1)) * g.nx + ((ix0 + a) & (g.nx - 1))] ==
                            DISCOS_BC_DIRICHLET)
                        v = -v;
                    atomicAdd(&acc[(lz * ty + lys[b]) * tx + lxs[a]], v);
                }
            }
        }
    }
    __syncthreads();
    // store the tile (tile sizes known at compile time for full tiles: no divisions)
    auto store = [&](const int sx, const int sy) {
        for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
            const int lx = k % sx, ly = (k / sx) % sy, lz = k / (sx * sy);
            const int gi = x0 + lx, gj = y0 + ly, gk = z0 + lz;
            double v = acc[k];
            if (add_bc && (gk == 0 || gk == g.nz - 1)) {
                for (int w = 0; w < 2; ++w) {
                    if (gk != (w == 0 ? 0 : g.nz - 1)) continue;
                    const double bv = wall.value[w] ? wall.value[w][(size_t)gj * g.nx + gi] : 0.0;
                    v += (wall_type_at(wall, w, gi, gj, g.nx) == DISCOS_BC_DIRICHLET)
                             ? 2.0 * wall.eps * bv * g.inv_h * g.inv_h
                             : bv * g.inv_h;
                }
            }
            out[((size_t)gk * g.ny + gj) * g.nx + gi] = v;
        }
    };
    if (tx == T && ty == T)
        store(T, T);
    else
        store(tx, ty);
}

template <bool MIXED>
__global__ void __launch_bounds__(SP_THREADS_ONE)
spread_charge_kernel(GridDev g, const double4* __restrict__ sxyzq, const int* __restrict__ bin_start,
                     double sign_lo, double sign_hi, int add_bc, WallDev wall,
                     double* __restrict__ out, int* __restrict__ flags) {
    __shared__ double acc[SP_TX * SP_TY * SP_TZ];
    __shared__ int rstart[SP_MAXR_ONE], rpre[SP_MAXR_ONE + 1], scan[SP_THREADS_ONE];
    const int tx = min(SP_TX, g.nx), ty = min(SP_TY, g.ny);
    int bx, by, bz;
    xcd_block3(bx, by, bz);
    spread_tile<SP_TX, MIXED, SP_TZ, SP_MAXR_ONE>(g, sxyzq, bin_start, sign_lo, sign_hi, add_bc, wall, out, bx * tx,
                              by * ty, bz * SP_TZ, acc, rstart, rpre, scan, flags);
}

// Batched: a persistent grid walks the (channel, tile) tasks; each channel's bins,
// cells and walls come from its descriptor.  The tile index runs x fastest over the
// channel's (nx / tx) x (ny / ty) x ceil(nz / T) tiles.
template <int T>
__global__ void __launch_bounds__(SP_THREADS)
spread_charge_batch_kernel(const RepDev* __restrict__ reps, const int2* __restrict__ tasks,
                           int ntasks, const double4* __restrict__ sxyzq,
                           const int* __restrict__ bin_start, double* __restrict__ out,
                           const int* __restrict__ sdirect, int* __restrict__ flags) {
    __shared__ double acc[T * T * T];
    __shared__ int rstart[SP_MAXR], rpre[SP_MAXR + 1], scan[SP_THREADS];
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const int2 task = tasks[t];
        const RepDev& R = reps[task.x];
        const GridDev g = R.g;
        const int tx = min(T, g.nx), ty = min(T, g.ny);
        const int ntx = g.nx / tx, nty = g.ny / ty;
        const int k = task.y;
        spread_tile<T>(g, sxyzq, bin_start + R.bin_off, R.s_lo, R.s_hi, 1, R.w, out + R.cell_off,
                       (k % ntx) * tx, ((k / ntx) % nty) * ty, (k / (ntx * nty)) * T, acc, rstart,
                       rpre, scan, flags, !sdirect[task.x]);
        __syncthreads();
    }
}

// Batched, the channels flagged in sdirect (few ions per tile): after the tile pass has
// stored their wall terms, one thread per ion adds its 4^3 window with global atomics.
__global__ void __launch_bounds__(256)
spread_charge_direct_batch_kernel(const RepDev* __restrict__ reps, const int* __restrict__ ion_rep,
                                  const int* __restrict__ sdirect, int n,
                                  const double4* __restrict__ sxyzq, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = ion_rep[i];
    if (!sdirect[r]) return;
    const RepDev& R = reps[r];
    const GridDev& g = R.g;
    const double4 a4 = sxyzq[i];
    if (!pos_ok(g, a4.x, a4.y, a4.z)) return;  // flagged by the interpolation
    int ix0, iy0, iz0;
    double wx[4], wy[4], wz[4];
    peskin4(a4.x * g.inv_h - 0.5, ix0, wx);
    peskin4(a4.y * g.inv_h - 0.5, iy0, wy);
    peskin4(a4.z * g.inv_h - 0.5, iz0, wz);
    const double scale = a4.w * g.inv_h * g.inv_h * g.inv_h;
    double* o = out + R.cell_off;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int kz = iz0 + c;
        double sgn = 1.0;
        if (kz < 0) {
            kz = -1 - kz;
            sgn = R.s_lo;
        } else if (kz >= g.nz) {
            kz = 2 * g.nz - 1 - kz;
            sgn = R.s_hi;
        }
        const double wzc = scale * sgn * wz[c];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const double wyz = wzc * wy[b];
            double* row = o + ((size_t)kz * g.ny + ((iy0 + b) & (g.ny - 1))) * g.nx;
#pragma unroll
            for (int a = 0; a < 4; ++a) atomicAdd(&row[(ix0 + a) & (g.nx - 1)], wyz * wx[a]);
        }
    }
}

int spread_charge_sorted(Ctx* c, const discos_params* p, int add_bc, double* out, hipStream_t s) {
    const GridDev& g = c->gd;
    const int tx = std::min(SP_TX, g.nx), ty = std::min(SP_TY, g.ny);
    dim3 grid(g.nx / tx, g.ny / ty, (g.nz + SP_TZ - 1) / SP_TZ);
    const double s_lo = p->bc_type[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    const double s_hi = p->bc_type[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    const WallDev w = wall_of(p);
    if (w.map[0] || w.map[1])
        spread_charge_kernel<true><<<grid, SP_THREADS_ONE, 0, s>>>(g, c->sxyzq, c->bin_start, s_lo, s_hi,
                                                               add_bc, w, out, c->flags);
    else
        spread_charge_kernel<false><<<grid, SP_THREADS_ONE, 0, s>>>(g, c->sxyzq, c->bin_start, s_lo, s_hi,
                                                                add_bc, w, out, c->flags);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int batch_spread(Batch* b, hipStream_t s) {
    const int v = b->cfg.spread_t == 8 ? 0 : 1;
    const int nt = b->ntasks[0][v];
    if (nt == 0) return DISCOS_OK;
    const int nb = b->cfg.spread_blocks > 0 ? std::min(nt, b->cfg.spread_blocks) : nt;
    if (v == 0)
        spread_charge_batch_kernel<8><<<nb, SP_THREADS, 0, s>>>(b->reps_d, b->tasks[0][0], nt,
                                                               b->sxyzq, b->bin_start, b->rho,
                                                               b->sdirect, b->flags);
    else
        spread_charge_batch_kernel<16><<<nb, SP_THREADS, 0, s>>>(b->reps_d, b->tasks[0][1], nt,
                                                                b->sxyzq, b->bin_start, b->rho,
                                                                b->sdirect, b->flags);
    if (b->n_sdirect > 0)
        spread_charge_direct_batch_kernel<<<(int)((b->n_tot + 255) / 256), 256, 0, s>>>(
            b->reps_d, b->ion_rep, b->sdirect, (int)b->n_tot, b->sxyzq, b->rho);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
