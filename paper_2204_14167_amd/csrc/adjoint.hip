// Energy U and electro-osmotic flux Q of the electrostatic pass (Sec. II.B.1, Sec. II.D
// stages 1-2) and their vector-Jacobian product, a hand-written adjoint:
//
//   rho = S q + b,  phi = A^+ rho,  E_i = J^es(-grad_h phi_ext)(x_i),
//   U = (1/2) dV <rho, phi>,   Q = sum_i w(z_i) q_i (E_x,i + E_ext,x),
//
// A = -eps lap_h with homogeneous ghosts (symmetric), b the wall terms, phi_ext the
// ghost-extended potential.  w(z) is the channel-mean x velocity per unit x force at
// height z from the kappa = 0 no-slip Stokes mode: with -eta D_zz g = 1 / nz and the
// no-slip ghosts, g_k = (z_k (Lz - z_k) + h^2 / 4) / (2 eta nz) exactly (z_k the cell
// heights), and w(z) = sum_k s_k g_k wz_k(z) / (nx ny h^3) with the no-slip image
// signs s.
//
// Reverse sweep for cotangents (gU, gQ):
//   lambda_i = gQ w_i q_i on E_x,i  ->  transposed E_x gather (onto x-faces with the
//   face weights, then the transposed face difference; ghost folds, and the ghost
//   layers' dependence on the wall fields gives part of their gradient)  ->  mu = A^+ lambda_phi (one Poisson solve)  ->  rbar = gU dV phi + mu,
//   the cotangent of rho  ->  per ion: dq = (J rbar)/dV + gQ w (E_x + E_ext,x),
//   dx = q grad(J rbar)/dV + gQ w q grad E_x + gQ F_x w'(z) e_z  (J with the
//   homogeneous folds of S);  wall fields: B^T rbar + ghost part;  dE_ext,x = gQ sum q w.
#include "kernels.h"

namespace discos {

// 4-point Peskin weights (as peskin4) and their derivatives d w / d s.
__device__ __forceinline__ void peskin4_d(double s, int& i0, double w[4], double dw[4]) {
    const double fl = floor(s);
    const double r = s - fl;
    const double q = sqrt(1.0 + 4.0 * r - 4.0 * r * r);
    const double dq = (2.0 - 4.0 * r) / q;
    i0 = (int)fl - 1;
    w[0] = (3.0 - 2.0 * r - q) * 0.125;
    w[1] = (3.0 - 2.0 * r + q) * 0.125;
    w[2] = (1.0 + 2.0 * r + q) * 0.125;
    w[3] = (1.0 + 2.0 * r - q) * 0.125;
    dw[0] = (-2.0 - dq) * 0.125;
    dw[1] = (-2.0 + dq) * 0.125;
    dw[2] = (2.0 + dq) * 0.125;
    dw[3] = (2.0 - dq) * 0.125;
}

struct FluxDev {
    double norm;       // 1 / (nx ny h^3)
    double inv2etanz;  // 1 / (2 eta nz)
};

// w(z) and dw/dz.
__device__ __forceinline__ void flux_weight(const GridDev& g, const FluxDev& f, double z, double& w,
                                            double& dw) {
    int i0;
    double wz[4], dz[4];
    peskin4_d(z * g.inv_h - 0.5, i0, wz, dz);
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int k = i0 + c;
        double s = 1.0;
        if (k < 0) { k = -1 - k; s = -1.0; }
        else if (k >= g.nz) { k = 2 * g.nz - 1 - k; s = -1.0; }
        const double zk = (k + 0.5) * g.h;
        const double gk = s * (zk * (g.Lz - zk) + 0.25 * g.h * g.h) * f.inv2etanz;
        a += gk * wz[c];
        b += gk * dz[c];
    }
    w = f.norm * a;
    dw = f.norm * b * g.inv_h;
}

// ---- deterministic reductions (fixed grid, fixed order) ---------------------------
#define RD_THREADS 256

__device__ __forceinline__ void block_sum_store(double v, double* out) {
    __shared__ double red[RD_THREADS];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = RD_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void __launch_bounds__(RD_THREADS)
dot_partials_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                    double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)RD_THREADS + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * RD_THREADS)
        acc += a[k] * b[k];
    block_sum_store(acc, part + blockIdx.x);
}

// sum_i w(z_i) v_i with v the sorted x forces (fx) or, with fx null, the charges; with
// part_q also sum_i w(z_i) q_i (the gradient of Q in E_ext, kept for the backward pass).
__global__ void __launch_bounds__(RD_THREADS)
flux_partials_kernel(GridDev g, FluxDev f, const double4* __restrict__ sxyzq,
                     const double* __restrict__ fx, int n, double* __restrict__ part,
                     double* __restrict__ part_q) {
    double acc = 0.0, accq = 0.0;
    for (int i = blockIdx.x * RD_THREADS + threadIdx.x; i < n; i += gridDim.x * RD_THREADS) {
        const double4 a4 = sxyzq[i];
        if (!pos_ok(g, a4.x, a4.y, a4.z)) continue;
        double w, dw;
        flux_weight(g, f, a4.z, w, dw);
        acc += w * (fx ? fx[i] : a4.w);
        accq += w * a4.w;
    }
    block_sum_store(acc, part + blockIdx.x);
    if (part_q) {
        __syncthreads();  // the block sum's LDS is reused
        block_sum_store(accq, part_q + blockIdx.x);
    }
}

// out[0] = scale (* mul[0] if given) * sum(part); with zero_tail also out[1] = out[2] = 0.
__global__ void __launch_bounds__(RD_THREADS)
finish_kernel(const double* __restrict__ part, int nparts, double scale, const double* __restrict__ mul,
              int zero_tail, double* __restrict__ out) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < nparts; k += RD_THREADS) acc += part[k];
    __shared__ double tot;
    block_sum_store(acc, &tot);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = scale * (mul ? mul[0] : 1.0) * tot;
        if (zero_tail) {
            out[1] = 0.0;
            out[2] = 0.0;
        }
    }
}

static int nparts_for(int64_t n) {
    const int64_t b = (n + RD_THREADS - 1) / RD_THREADS;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, PART_MAX));
}

// ---- transposed E_x gather: lambda_i = gQ w_i q_i onto the cell grid --------------
#define AS_T 16   // tile edge in x and y
#define AS_TZ 16  // tile edge in z
#define AS_THREADS 512
#define AS_MAXR 256

__global__ void __launch_bounds__(AS_THREADS)
flux_lambda_kernel(GridDev g, WallDev wl, FluxDev f, const double4* __restrict__ sxyzq,
                   const int* __restrict__ bin_start, const double* __restrict__ gvec,
                   double* __restrict__ lam, double* __restrict__ bcg, int* __restrict__ flags) {
    // mu on the x-faces x0 .. x0 + tx of the tile (face F between cells F - 1 and F), then
    // lambda_phi(cell c) = mu(c) - mu(c + 1): the transpose of the face differences
    constexpr int FX = AS_T + 1;
    __shared__ double acc[FX * AS_T * AS_TZ];
    __shared__ double glo[FX * AS_T], ghi[FX * AS_T];
    __shared__ int rstart[AS_MAXR], rpre[AS_MAXR + 1], scan[AS_THREADS];
    const int tx = min(AS_T, g.nx), ty = min(AS_T, g.ny);
    const int fx = tx + 1;  // face columns held (face x0 + tx is face x0 when tx = nx)
    int bx, by, bz;
    xcd_block3(bx, by, bz);
    const int x0 = bx * tx, y0 = by * ty, z0 = bz * AS_TZ;
    const int tz = min(AS_TZ, g.nz - z0);
    const bool has_lo = z0 == 0, has_hi = z0 + tz == g.nz;
    for (int k = threadIdx.x; k < fx * ty * tz; k += blockDim.x) acc[k] = 0.0;
    for (int k = threadIdx.x; k < fx * ty; k += blockDim.x) glo[k] = ghi[k] = 0.0;
    static_assert(tile_rows_bound(AS_T, AS_TZ, 2, 2) <= AS_MAXR, "adjoint tile rows exceed AS_MAXR");
    const int nr = tile_ranges<AS_MAXR>(g, bin_start, x0, y0, z0, tx, ty, tz, rstart, rpre, scan,
                                        flags);
    const int total = rpre[nr];
    const double gQ = gvec[1];
    const double s_lo = wl.type[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    const double s_hi = wl.type[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    auto ion_at = [&](int e) {
        int r = 0, hi = nr - 1;
        while (r < hi) {
            const int mid = (r + hi + 1) >> 1;
            if (rpre[mid] <= e) r = mid; else hi = mid - 1;
        }
        return sxyzq[rstart[r] + (e - rpre[r])];
    };
    // the next ion's record is loaded before the current one's LDS atomics
    double4 nxt = make_double4(0.0, 0.0, 0.0, 0.0);
    if ((int)threadIdx.x < total) nxt = ion_at(threadIdx.x);
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const double4 a4 = nxt;
        if (e + (int)blockDim.x < total) nxt = ion_at(e + blockDim.x);
        if (!pos_ok(g, a4.x, a4.y, a4.z)) continue;
        double w, dw;
        flux_weight(g, f, a4.z, w, dw);
        const double val = -gQ * w * a4.w * g.inv_h;
        if (val == 0.0) continue;
        int ifx, icy, icz;
        double wfx[4], wcy[4], wcz[4];
        peskin4(a4.x * g.inv_h, ifx, wfx);
        peskin4(a4.y * g.inv_h - 0.5, icy, wcy);
        peskin4(a4.z * g.inv_h - 0.5, icz, wcz);
        int lfs[4], lys[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            lfs[q] = (ifx + q - x0) & (g.nx - 1);
            lys[q] = (icy + q - y0) & (g.ny - 1);
        }
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
            const int k = icz + c;
            int layer = k, m = -1, wall = -1;
            double sg = 1.0;
            if (k < 0) { m = -1 - k; layer = m; sg = s_lo; wall = 0; }
            else if (k >= g.nz) { m = k - g.nz; layer = g.nz - 1 - m; sg = s_hi; wall = 1; }
            const int lz = layer - z0;
            const bool in_z = lz >= 0 && lz < tz;
            // the ghost layer's dependence on the wall field: 2 (Dirichlet) or
            // (2m+1) h / eps (Neumann) per unit of the column's value
            const bool ghost = (wall == 0 && has_lo) || (wall == 1 && has_hi);
            double gcoef = 0.0;
            if (ghost)
                gcoef = wl.type[wall] == DISCOS_BC_DIRICHLET ? 2.0 : (2 * m + 1) * g.h / wl.eps;
            if (!in_z && !ghost) continue;
            double* gl = wall == 0 ? glo : ghi;
            const double vz = val * wcz[c];
#pragma unroll
            for (int bq = 0; bq < 4; ++bq) {
                const int ly = lys[bq];
                if (ly >= ty) continue;
                const double vyz = vz * wcy[bq];
#pragma unroll
                for (int aq = 0; aq < 4; ++aq) {
                    const int lf = lfs[aq];
                    if (lf >= fx) continue;
                    const double v = vyz * wfx[aq];
                    if (in_z) atomicAdd(&acc[(lz * ty + ly) * fx + lf], sg * v);
                    if (ghost) atomicAdd(&gl[ly * fx + lf], gcoef * v);
                }
            }
        }
    }
    __syncthreads();
    // store lambda_phi = mu(c) - mu(c + 1) per cell (and the same difference of the ghost
    // parts per wall column); tile sizes known at compile time for full tiles
    const bool wrap = tx == g.nx;  // the face after the last cell is face 0
    auto store = [&](const int sx, const int sy) {
        for (int k = threadIdx.x; k < sx * sy * tz; k += blockDim.x) {
            const int lx = k % sx, ly = (k / sx) % sy, lz = k / (sx * sy);
            const int nx1 = (wrap && lx == sx - 1) ? 0 : lx + 1;
            const int row = (lz * sy + ly) * fx;
            lam[((size_t)(z0 + lz) * g.ny + (y0 + ly)) * g.nx + (x0 + lx)] = acc[row + lx] - acc[row + nx1];
        }
        if (has_lo || has_hi)
            for (int k = threadIdx.x; k < sx * sy; k += blockDim.x) {
                const int lx = k % sx, ly = k / sx;
                const int nx1 = (wrap && lx == sx - 1) ? 0 : lx + 1;
                const size_t col = (size_t)(y0 + ly) * g.nx + (x0 + lx);
                if (has_lo) bcg[col] = glo[ly * fx + lx] - glo[ly * fx + nx1];
                if (has_hi) bcg[(size_t)g.nx * g.ny + col] = ghi[ly * fx + lx] - ghi[ly * fx + nx1];
            }
    };
    if (tx == AS_T && ty == AS_T)
        store(AS_T, AS_T);
    else
        store(tx, ty);
}

// ---- per-ion gradients: gather of rbar (homogeneous folds) on the centre window and of
// the x-face differences of phi_ext (wall ghosts) on the face window ------------------
// 16^3 tiles: the two staged arrays with their halos fill most of the LDS, so one
// workgroup runs per CU; 12 wavefronts of it take the tile's ions (about 512 at the
// densities of the workloads) and the staging
#define GT_TX 16
#define GT_TY 16
#define GT_TZ 16
#define GT_H 5
#define GT_THREADS 768
#define GT_MAXR 64  // bin rows of a tile: 8 z slabs x 8 y rows
#define GT_UNROLL 4  // staging elements in flight per thread

__global__ void __launch_bounds__(GT_THREADS)
flux_energy_grad_kernel(GridDev g, WallDev wl, FluxDev f, const double4* __restrict__ sxyzq,
                        const int* __restrict__ bin_start, const int* __restrict__ perm,
                        const double* __restrict__ phi, const double* __restrict__ mu,
                        const double* __restrict__ gvec, double ex0, double* __restrict__ dpos,
                        double* __restrict__ dq, int64_t stride, int* __restrict__ flags) {
    constexpr int LX = GT_TX + GT_H, LY = GT_TY + GT_H, LZ = GT_TZ + GT_H;
    __shared__ double trb[LZ * LY * LX];
    __shared__ double tph[LZ * LY * LX];
    __shared__ int rstart[GT_MAXR], rpre[GT_MAXR + 1], scan[GT_THREADS];
    const int tx = min(GT_TX, g.nx), ty = min(GT_TY, g.ny);
    int bx, by, bz;
    xcd_block3(bx, by, bz);  // neighbouring tiles, whose halos overlap, on one XCD
    const int x0 = bx * tx, y0 = by * ty, z0 = bz * GT_TZ;
    const int tz = min(GT_TZ, g.nz - z0);
    const int lxn = tx + GT_H, lyn = ty + GT_H, lzn = tz + GT_H;
    const double dV = g.h * g.h * g.h;
    const double gU = gvec[0], gQ = gvec[1];
    const double udv = gU * dV;
    const double s_lo = wl.type[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    const double s_hi = wl.type[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    const int nbxt = tx >> g.lb, nbyt = ty >> g.lb;
    const int bz0 = z0 >> g.lb, bz1 = (z0 + tz - 1) >> g.lb;
    static_assert((GT_TZ / DISCOS_BIN) * (GT_TY / DISCOS_BIN) <= GT_MAXR && GT_MAXR <= GT_THREADS,
                  "gradient tile rows exceed GT_MAXR");
    const int nrows = (bz1 - bz0 + 1) * nbyt;
    const int ne = LX * LY * lzn;
    const bool inner = z0 >= 2 && z0 + tz + 3 <= g.nz;  // no ghost layer in the window
    // an inner tile's window (every element of this thread) is loaded before the row scan,
    // so that its loads and the bin-start loads are in flight together
    constexpr int NPT = (LX * LY * LZ + GT_THREADS - 1) / GT_THREADS;
    double er[NPT], ep[NPT];
    if (inner) {
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int e = threadIdx.x + u * GT_THREADS;
            const int lx = e % LX, ly = (e / LX) % LY, lz = e / (LX * LY);
            const int i = (x0 - 2 + lx) & (g.nx - 1), j = (y0 - 2 + ly) & (g.ny - 1);
            const int il = (i - 1) & (g.nx - 1);
            er[u] = 0.0;
            ep[u] = 0.0;
            if (e < ne && lx < lxn && ly < lyn) {
                const size_t row = ((size_t)(z0 - 2 + lz) * g.ny + j) * g.nx;
                const double pv = phi[row + i];
                er[u] = udv * pv + mu[row + i];
                ep[u] = pv - phi[row + il];
            }
        }
    }
    {
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
    if (rpre[nrows] == 0) return;  // the same for the whole workgroup
    // rbar (homogeneous folds) and phi (wall ghosts) on the tile and its halo; GT_UNROLL
    // elements per thread are loaded before the first LDS store
    if (inner) {
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int e = threadIdx.x + u * GT_THREADS;
            if (e < ne) {
                trb[e] = er[u];
                tph[e] = ep[u];
            }
        }
    }
    for (int e0 = threadIdx.x; !inner && e0 < ne; e0 += GT_UNROLL * GT_THREADS) {
        double vr[GT_UNROLL], vp[GT_UNROLL];
#pragma unroll
        for (int u = 0; u < GT_UNROLL; ++u) {
            const int e = e0 + u * GT_THREADS;
            const int lx = e % LX, ly = (e / LX) % LY, lz = e / (LX * LY);
            const int i = (x0 - 2 + lx) & (g.nx - 1), j = (y0 - 2 + ly) & (g.ny - 1);
            const int k = z0 - 2 + lz;
            const int il = (i - 1) & (g.nx - 1);  // left neighbour: face i lies between il and i
            vr[u] = 0.0;
            vp[u] = 0.0;
            if (e < ne && lx < lxn && ly < lyn) {
                if (inner) {
                    const size_t row = ((size_t)k * g.ny + j) * g.nx;
                    const double pv = phi[row + i];
                    vr[u] = udv * pv + mu[row + i];
                    vp[u] = pv - phi[row + il];
                } else {
                    int src = k;
                    double sg = 1.0;
                    if (k < 0) { src = -1 - k; sg = s_lo; }
                    else if (k >= g.nz) { src = 2 * g.nz - 1 - k; sg = s_hi; }
                    src = min(max(src, 0), g.nz - 1);
                    const size_t o = ((size_t)src * g.ny + j) * g.nx + i;
                    vr[u] = sg * (udv * phi[o] + mu[o]);
                    vp[u] = phi_at(phi, g, wl, i, j, k) - phi_at(phi, g, wl, il, j, k);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < GT_UNROLL; ++u) {
            const int e = e0 + u * GT_THREADS;
            if (e < ne) {
                trb[e] = vr[u];
                tph[e] = vp[u];
            }
        }
    }
    __syncthreads();
    const int total = rpre[nrows];
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        int r = 0, hi = nrows - 1;
        while (r < hi) {
            const int mid = (r + hi + 1) >> 1;
            if (rpre[mid] <= e) r = mid; else hi = mid - 1;
        }
        const int i = rstart[r] + (e - rpre[r]);
        const int o = perm[i];
        const double4 a4 = sxyzq[i];
        bool ok = pos_ok(g, a4.x, a4.y, a4.z);
        // centre weights (and d/du) in x, y, z; face weights (and d/du) in x
        double wcx[4], dcx[4], wfx[4], dfx[4], wcy[4], dcy[4], wcz[4], dcz[4];
        int ax = 0, dx0 = 0, ay = 0, az = 0;  // tile indices of the window starts
        if (ok) {
            const double ux = a4.x * g.inv_h, uy = a4.y * g.inv_h, uz = a4.z * g.inv_h;
            int icx, ifx, icy, icz;
            peskin4_d(ux - 0.5, icx, wcx, dcx);
            peskin4_d(ux, ifx, wfx, dfx);
            peskin4_d(uy - 0.5, icy, wcy, dcy);
            peskin4_d(uz - 0.5, icz, wcz, dcz);
            const int cx = ifx + 1, cy = (int)floor(uy), cz = (int)floor(uz);
            const int lx0 = (cx - x0) & (g.nx - 1);
            const int ly0 = (cy - y0) & (g.ny - 1);
            const int lz0 = cz - z0;
            ok = lx0 <= tx && ly0 <= ty && lz0 >= 0 && lz0 <= tz;
            // the tile starts at cell x0 - 2; faces F (between cells F - 1 and F) are
            // stored at the index of cell F
            ax = lx0 + (icx - (cx - 2));
            dx0 = lx0 + 1;
            ay = ly0 + (icy - (cy - 2));
            az = lz0 + (icz - (cz - 2));
        }
        if (!ok) {
            set_flag(flags, (isfinite(a4.x) && isfinite(a4.y) && isfinite(a4.z)) ? DISCOS_FLAG_OUT_OF_DOMAIN
                                                                              : DISCOS_FLAG_NONFINITE);
            if (dq) dq[o] = 0.0;
            if (dpos) dpos[o] = dpos[o + stride] = dpos[o + 2 * stride] = 0.0;
            continue;
        }
        // R = J rbar and its gradient (4^3 centre window); P = sum wf_x wc_y wc_z D (the
        // x-face differences of phi_ext, 4^3 window) and its gradient
        double R = 0.0, Rx = 0.0, Ry = 0.0, Rz = 0.0, P = 0.0, Px = 0.0, Py = 0.0, Pz = 0.0;
#pragma unroll 1
        for (int c = 0; c < 4; ++c) {
            double c00 = 0.0, c10 = 0.0, c01 = 0.0, e00 = 0.0, e10 = 0.0, e01 = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int rowc = ((az + c) * LY + ay + b) * LX;
                const double* ra = &trb[rowc + ax];
                const double* rd = &tph[rowc + dx0];
                double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const double rv = ra[a], dv = rd[a];
                    a0 += wcx[a] * rv;
                    a1 += dcx[a] * rv;
                    b0 += wfx[a] * dv;
                    b1 += dfx[a] * dv;
                }
                c00 += wcy[b] * a0;
                c10 += wcy[b] * a1;
                c01 += dcy[b] * a0;
                e00 += wcy[b] * b0;
                e10 += wcy[b] * b1;
                e01 += dcy[b] * b0;
            }
            R += wcz[c] * c00;
            Rx += wcz[c] * c10;
            Ry += wcz[c] * c01;
            Rz += dcz[c] * c00;
            P += wcz[c] * e00;
            Px += wcz[c] * e10;
            Py += wcz[c] * e01;
            Pz += dcz[c] * e00;
        }
        const double ih = g.inv_h;
        const double Ex = -ih * P;
        double w, dw;
        flux_weight(g, f, a4.z, w, dw);
        const double qi = a4.w;
        const double Fx = qi * (Ex + ex0);
        const double gwq = gQ * w * qi;
        if (dq) dq[o] = R / dV + gQ * w * (Ex + ex0);
        if (dpos) {
            const double s = qi * ih / dV;
            const double e2 = -ih * ih;
            dpos[o] = s * Rx + gwq * e2 * Px;
            dpos[o + stride] = s * Ry + gwq * e2 * Py;
            dpos[o + 2 * stride] = s * Rz + gwq * e2 * Pz + gQ * dw * Fx;
        }
    }
}

// Wall-field gradients: B^T rbar on the end layers plus the ghost-layer part.
__global__ void flux_bc_kernel(GridDev g, WallDev wl, const double* __restrict__ phi,
                               const double* __restrict__ mu, const double* __restrict__ gvec,
                               const double* __restrict__ bcg, double* __restrict__ dlo,
                               double* __restrict__ dhi) {
    const int64_t ncol = (int64_t)g.nx * g.ny;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ncol) return;
    const double udv = gvec[0] * g.h * g.h * g.h;
    for (int wall = 0; wall < 2; ++wall) {
        double* d = wall == 0 ? dlo : dhi;
        if (!d) continue;
        const size_t o = (size_t)(wall == 0 ? 0 : g.nz - 1) * ncol + t;
        const double coef = wl.type[wall] == DISCOS_BC_DIRICHLET ? 2.0 * wl.eps * g.inv_h * g.inv_h : g.inv_h;
        d[t] = coef * (udv * phi[o] + mu[o]) + bcg[wall * ncol + t];
    }
}

static FluxDev flux_of(const Ctx* c, const discos_params* p) {
    FluxDev f;
    const double h = c->grid.h;
    f.norm = 1.0 / ((double)c->grid.nx * c->grid.ny * h * h * h);
    f.inv2etanz = 1.0 / (2.0 * p->eta * c->grid.nz);
    return f;
}

int energy_flux(Ctx* c, int n, const discos_params* p, const double* phi, double* out, hipStream_t s) {
    // U = (1/2) dV <rho, phi> (c->rho holds S q + b), Q = sum w(z) F_x (c->fp sorted)
    const double dV = c->grid.h * c->grid.h * c->grid.h;
    const int pu = nparts_for(c->ncell);
    dot_partials_kernel<<<pu, RD_THREADS, 0, s>>>(c->rho, phi, c->ncell, c->part);
    finish_kernel<<<1, RD_THREADS, 0, s>>>(c->part, pu, 0.5 * dV, nullptr, 0, out);
    const int pq = nparts_for(n);
    const FluxDev f = flux_of(c, p);
    flux_partials_kernel<<<pq, RD_THREADS, 0, s>>>(c->gd, f, c->sxyzq, c->fp, n, c->part + PART_MAX,
                                                   c->part + 2 * PART_MAX);
    finish_kernel<<<1, RD_THREADS, 0, s>>>(c->part + PART_MAX, pq, 1.0, nullptr, 0, out + 1);
    c->ef_wq = f.inv2etanz;  // the partials of sum w q held for this flux weight
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int energy_flux_backward(Ctx* c, int n, const discos_params* p, const double* phi, const double* gvec,
                         double* dpos, double* dq, double* dlo, double* dhi, double* de, bool reuse,
                         hipStream_t s) {
    const GridDev& g = c->gd;
    const FluxDev f = flux_of(c, p);
    const WallDev wl = wall_of(p);
    // lambda_phi -> c->rho, wall ghost part -> c->bcg
    dim3 ga(g.nx / std::min(AS_T, g.nx), g.ny / std::min(AS_T, g.ny), (g.nz + AS_TZ - 1) / AS_TZ);
    flux_lambda_kernel<<<ga, AS_THREADS, 0, s>>>(g, wl, f, c->sxyzq, c->bin_start, gvec, c->rho, c->bcg,
                                                 c->flags);
    // mu = A^+ lambda_phi -> c->phi
    int rc = solve_poisson(c, c->rho, p, c->phi, s, -1, 1);
    if (rc) return rc;
    if (n > 0 && (dpos || dq)) {
        dim3 gg(g.nx / std::min(GT_TX, g.nx), g.ny / std::min(GT_TY, g.ny), (g.nz + GT_TZ - 1) / GT_TZ);
        flux_energy_grad_kernel<<<gg, GT_THREADS, 0, s>>>(g, wl, f, c->sxyzq, c->bin_start, c->perm, phi,
                                                         c->phi, gvec, p->e_ext[0], dpos, dq, n, c->flags);
    }
    if (dlo || dhi) {
        const int64_t ncol = (int64_t)g.nx * g.ny;
        flux_bc_kernel<<<(int)((ncol + 255) / 256), 256, 0, s>>>(g, wl, phi, c->phi, gvec, c->bcg, dlo, dhi);
    }
    if (de) {
        // sum w q: from the forward pass when it ran on these cells with this weight
        const int pq = nparts_for(n);
        if (!(reuse && c->ef_wq == f.inv2etanz))
            flux_partials_kernel<<<pq, RD_THREADS, 0, s>>>(g, f, c->sxyzq, nullptr, n,
                                                           c->part + 2 * PART_MAX, nullptr);
        finish_kernel<<<1, RD_THREADS, 0, s>>>(c->part + 2 * PART_MAX, pq, 1.0, gvec + 1, 1, de);
    }
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
