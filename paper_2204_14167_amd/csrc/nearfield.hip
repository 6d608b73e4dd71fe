// Particle-particle part of the step: the P3M near-field correction with wall images
// (eqs coulomb, fullElectro, LC and the image rule of Sec. II.B.1), the 9-3 wall
// force and the optional ion-ion LJ force (Sec. II.B.2), and the dry update
// (eq ions3, eq step2 with the tensor of eq diff1).  One thread per ion in cell-list
// order; neighbours come from the (2R+1)^2 rows of 2R+1 contiguous bins around the
// ion's bin, so consecutive threads read overlapping, cache-resident neighbour lists.
#include "kernels.h"

namespace discos {

struct NearDev {
    double psi, psi2g, inv4pieps, h, inv_h2, inv_hdr;
    double rsearch;  // search radius: psi, or the LJ range if larger
    const double* tab;
    int tablen;
    int R;  // search radius in bins
    double s_lo, s_hi;
    int wall_on;
    double wsig, wxi, wcut;
    int lj_on;
    const double* ljs;
    const double* ljx;
    double ljf;
    int nsp;
};

static NearDev near_of(const Ctx* c, const discos_params* p) {
    NearDev d;
    d.psi = p->psi;
    d.psi2g = p->psi * p->psi * (1.0 + 1e-12);
    d.inv4pieps = 1.0 / (4.0 * M_PI * p->eps);
    d.h = c->grid.h;
    d.inv_h2 = 1.0 / (c->grid.h * c->grid.h);
    d.inv_hdr = 1.0 / (c->grid.h * p->p3m_dr);
    d.tab = p->p3m_table;
    d.tablen = p->p3m_len;
    double range = p->psi;
    if (p->lj_on) range = std::max(range, p->lj_range);
    d.rsearch = range;
    d.R = (int)std::ceil(range / (DISCOS_BIN * c->grid.h));
    d.s_lo = p->bc_type[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    d.s_hi = p->bc_type[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    d.wall_on = p->wall_on;
    d.wsig = p->wall_sigma;
    d.wxi = p->wall_xi;
    d.wcut = p->wall_cut;
    d.lj_on = p->lj_on;
    d.ljs = p->lj_sigma;
    d.ljx = p->lj_xi;
    d.ljf = p->lj_cut_factor;
    d.nsp = p->nspecies;
    return d;
}

int near_radius_bins(const Ctx* c, const discos_params* p) { return near_of(c, p).R; }

// F^C - F^P for one pair (or ion-image pair) at separation d, charge product qq.
// A pair at zero separation has no direction and contributes nothing.
__device__ __forceinline__ void es_pair(double dx, double dy, double dz, double qq,
                                        const NearDev& P, double& fx, double& fy, double& fz) {
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < P.psi2g) || !(r2 > 0.0)) return;
    const double r = sqrt(r2);
    if (!(r < P.psi)) return;
    const double inv_r = 1.0 / r;
    const double t = r * P.inv_hdr;
    int k = (int)t;
    const double f = t - k;
    k = min(k, P.tablen - 2);
    const double g0 = P.tab[k], g1 = P.tab[k + 1];
    const double gv = g0 * (1.0 - f) + g1 * f;
    const double mag = qq * P.inv4pieps * (inv_r * inv_r - gv * P.inv_h2) * inv_r;
    fx += mag * dx;
    fy += mag * dy;
    fz += mag * dz;
}

__device__ __forceinline__ void lj_pair(double dx, double dy, double dz, int si, int sj,
                                        const NearDev& P, double& fx, double& fy, double& fz) {
    if (si < 0 || si >= P.nsp || sj < 0 || sj >= P.nsp) return;  // flagged by the caller
    const double sig = P.ljs[si * P.nsp + sj];
    const double xi = P.ljx[si * P.nsp + sj];
    const double cut = P.ljf * sig;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < cut * cut * (1.0 + 1e-12))) return;
    const double r = sqrt(r2);
    if (!(r > 0.0 && r < cut)) return;
    const double du = 4.0 * xi * (-12.0 * pow(sig, 12.0) / pow(r, 13.0) + 6.0 * pow(sig, 6.0) / pow(r, 7.0));
    const double m = -du / r;
    fx += m * dx;
    fy += m * dy;
    fz += m * dz;
}

__device__ __forceinline__ double du93(double y, const NearDev& P) {
    if (!(y > 0.0 && y < P.wcut)) return 0.0;
    const double c93 = 1.5 * sqrt(3.0);
    return c93 * P.wxi * (-9.0 * pow(P.wsig, 9.0) / pow(y, 10.0) + 3.0 * pow(P.wsig, 3.0) / pow(y, 4.0));
}

// Near-field force on ion i (cell-list index) from the real ions within the search
// radius (mode 0) and from the wall images (modes 1: -z_j, 2: 2 Lz - z_j).  Rows of
// bins are visited in unwrapped coordinates around the ion; a row is skipped when its
// slab is farther than the search radius, and only the x-bins that can reach the
// sphere are read.  Periodic copies get an explicit shift of +-L, so no per-pair
// minimum-image arithmetic is needed (2R+1 <= nbx, nby is checked on the host).
__device__ void near_force(int i, double4 me, int spi, const double4* __restrict__ sxyzq,
                           const int* __restrict__ ssp, const int* __restrict__ bin_start,
                           const GridDev& g, const NearDev& P, double& Fx, double& Fy,
                           double& Fz) {
    const double xi = me.x, yi = me.y, zi = me.z, qi = me.w;
    const double Bh = DISCOS_BIN * g.h;
    const double inv_Bh = 1.0 / Bh;
    const double rs2 = P.rsearch * P.rsearch;
    int bx, by, bz;
    bin_of(g, xi, yi, zi, bx, by, bz);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int mode = 0; mode < 3; ++mode) {
        int zlo, zhi;
        double sgn = 1.0;
        if (mode == 0) {
            zlo = max(bz - P.R, 0);
            zhi = min(bz + P.R, g.nbz - 1);
        } else if (mode == 1) {
            if (!(zi < P.psi)) continue;
            zlo = 0;
            zhi = min(g.nbz - 1, (int)floor(P.psi * g.inv_h) / DISCOS_BIN);
            sgn = P.s_lo;
        } else {
            if (!(zi > g.Lz - P.psi)) continue;
            zlo = max(0, (int)floor((g.Lz - P.psi) * g.inv_h) / DISCOS_BIN);
            zhi = g.nbz - 1;
            sgn = P.s_hi;
        }
        const double r2m = mode == 0 ? rs2 : P.psi * P.psi;
        for (int cz = zlo; cz <= zhi; ++cz) {
            const double zb0 = cz * Bh, zb1 = fmin((cz + 1) * Bh, g.Lz);
            double dzm;
            if (mode == 0)
                dzm = fmax(0.0, fmax(zb0 - zi, zi - zb1));
            else if (mode == 1)
                dzm = zi + zb0;
            else
                dzm = (2.0 * g.Lz - zb1) - zi;
            const double remz = r2m - dzm * dzm;
            if (!(remz > 0.0)) continue;
            for (int dyb = -P.R; dyb <= P.R; ++dyb) {
                const int cyu = by + dyb;
                const double yb0 = cyu * Bh, yb1 = yb0 + Bh;
                const double dym = fmax(0.0, fmax(yb0 - yi, yi - yb1));
                const double rem = remz - dym * dym;
                if (!(rem > 0.0)) continue;
                const double wx = sqrt(rem);
                const int bxl = max(bx - P.R, (int)floor((xi - wx) * inv_Bh));
                const int bxh = min(bx + P.R, (int)floor((xi + wx) * inv_Bh));
                if (bxl > bxh) continue;
                const int cy = cyu < 0 ? cyu + g.nby : (cyu >= g.nby ? cyu - g.nby : cyu);
                const double shy = cyu < 0 ? -g.Ly : (cyu >= g.nby ? g.Ly : 0.0);
                const int row = (cz * g.nby + cy) * g.nbx;
                // split [bxl, bxh] into at most two wrapped segments
                int sa[2], sb[2];
                double shx[2];
                int nseg = 0;
                if (bxl < 0) {
                    sa[nseg] = bxl + g.nbx; sb[nseg] = g.nbx - 1; shx[nseg] = -g.Lx; ++nseg;
                    if (bxh >= 0) { sa[nseg] = 0; sb[nseg] = bxh; shx[nseg] = 0.0; ++nseg; }
                } else if (bxh >= g.nbx) {
                    if (bxl < g.nbx) { sa[nseg] = bxl; sb[nseg] = g.nbx - 1; shx[nseg] = 0.0; ++nseg; }
                    sa[nseg] = max(bxl - g.nbx, 0); sb[nseg] = bxh - g.nbx; shx[nseg] = g.Lx; ++nseg;
                } else {
                    sa[nseg] = bxl; sb[nseg] = bxh; shx[nseg] = 0.0; ++nseg;
                }
                for (int s = 0; s < nseg; ++s) {
                    const int j0 = bin_start[row + sa[s]], j1 = bin_start[row + sb[s] + 1];
                    const double xs = xi - shx[s], ys = yi - shy;
                    for (int j = j0; j < j1; ++j) {
                        const double4 o = sxyzq[j];
                        const double dx = xs - o.x;
                        const double dy = ys - o.y;
                        if (mode == 0) {
                            if (j == i) continue;
                            const double dz = zi - o.z;
                            es_pair(dx, dy, dz, qi * o.w, P, fx, fy, fz);
                            if (P.lj_on) lj_pair(dx, dy, dz, spi, ssp[j], P, fx, fy, fz);
                        } else {
                            const double zimg = mode == 1 ? -o.z : 2.0 * g.Lz - o.z;
                            es_pair(dx, dy, zi - zimg, qi * (sgn * o.w), P, fx, fy, fz);
                        }
                    }
                }
            }
        }
    }
    if (P.wall_on) fz += -du93(zi, P) + du93(g.Lz - zi, P);
    Fx = fx;
    Fy = fy;
    Fz = fz;
}

__global__ void near_field_kernel(GridDev g, NearDev P, int n, const double4* __restrict__ sxyzq,
                                  const int* __restrict__ ssp, const int* __restrict__ bin_start,
                                  const int* __restrict__ perm, double* __restrict__ out,
                                  int64_t stride, int scatter, int* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 me = sxyzq[i];
    if (!pos_ok(g, me.x, me.y, me.z)) return;
    double Fx, Fy, Fz;
    const int spi = P.lj_on ? ssp[i] : 0;
    if (spi < 0 || spi >= max(P.nsp, 1)) set_flag(flags, DISCOS_FLAG_BAD_SPECIES);
    near_force(i, me, spi, sxyzq, ssp, bin_start, g, P, Fx, Fy, Fz);
    const int o = scatter ? perm[i] : i;
    out[o] += Fx;
    out[o + stride] += Fy;
    out[o + 2 * stride] += Fz;
}

int near_field_sorted(Ctx* c, int n, const discos_params* p, double* out, int64_t out_stride,
                      int scatter_to_caller, hipStream_t s) {
    if (n <= 0) return DISCOS_OK;
    const int T = 128;
    near_field_kernel<<<(n + T - 1) / T, T, 0, s>>>(c->gd, near_of(c, p), n, c->sxyzq, c->ssp,
                                                    c->bin_start, c->perm, out, out_stride,
                                                    scatter_to_caller, c->flags);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

// ---- dry update --------------------------------------------------------------

struct DryDev {
    int nsp;
    double kT, eta, dt;
    const double* radius;
    const double* coef;  // [nsp][2][7]
    uint64_t seed, step;
};

__device__ __forceinline__ double gamma_hat(double y, const double* c) {
    const double t3 = c[4] + y, t5 = c[6] + y;
    return c[0] + c[1] / (c[2] + y) + c[3] / pow(t3, 3.0) + c[5] / pow(t5, 5.0);
}

__device__ __forceinline__ double dgamma_hat(double y, const double* c) {
    const double t1 = c[2] + y, t3 = c[4] + y, t5 = c[6] + y;
    return -c[1] / pow(t1, 2.0) - 3.0 * c[3] / pow(t3, 4.0) - 5.0 * c[5] / pow(t5, 6.0);
}

__device__ __forceinline__ double wrap_coord(double x, double L) {
    double r = fmod(x, L);
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

__global__ void force_update_dry_kernel(GridDev g, NearDev P, DryDev Dd, int n,
                                        const double4* __restrict__ sxyzq,
                                        const int* __restrict__ sid, const int* __restrict__ ssp,
                                        const int* __restrict__ bin_start,
                                        const double* __restrict__ fp, int64_t fstride,
                                        double* __restrict__ pos, int64_t pstride,
                                        double* __restrict__ q, int* __restrict__ id,
                                        int* __restrict__ sp, int* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 me = sxyzq[i];
    const double xi = me.x, yi = me.y, zi = me.z;
    const double qi = me.w;
    const int sp_in = ssp[i];
    const int idi = sid[i];
    const bool sp_ok = sp_in >= 0 && sp_in < Dd.nsp;
    if (!sp_ok) set_flag(flags, DISCOS_FLAG_BAD_SPECIES);
    const int spi = sp_ok ? sp_in : 0;
    double nx = xi, ny = yi, nz = zi;
    if (pos_ok(g, xi, yi, zi)) {
        double Fx, Fy, Fz;
        near_force(i, me, spi, sxyzq, ssp, bin_start, g, P, Fx, Fy, Fz);
        Fx += fp[i];
        Fy += fp[i + fstride];
        Fz += fp[i + 2 * fstride];
        const double a = Dd.radius[spi];
        const double D = Dd.kT / (6.0 * M_PI * Dd.eta * a);
        const double* cpar = Dd.coef + (size_t)spi * 14;
        const double* cperp = cpar + 7;
        const bool below = zi <= g.Lz - zi;
        const double yw = below ? zi : g.Lz - zi;
        const double gpar = gamma_hat(yw, cpar);
        const double gperp = gamma_hat(yw, cperp);
        const double Gp = fmin(fmax(gpar, 0.0), 1.0);
        const double Gn = fmin(fmax(gperp, 0.0), 1.0);
        const double dG = (gperp > 0.0 && gperp < 1.0) ? (below ? 1.0 : -1.0) * dgamma_hat(yw, cperp) : 0.0;
        double wx, wy, wz, wunused;
        normal_pair(Dd.seed, Dd.step, DISCOS_TAG_DRY, 0u, (uint32_t)idi, wx, wy);
        normal_pair(Dd.seed, Dd.step, DISCOS_TAG_DRY, 1u, (uint32_t)idi, wz, wunused);
        const double dtD = Dd.dt * D;
        double dx = dtD * Gp * Fx / Dd.kT;
        double dy = dtD * Gp * Fy / Dd.kT;
        double dz = dtD * Gn * Fz / Dd.kT;
        dz += dtD * dG;
        dx += sqrt(2.0 * D * Gp * Dd.dt) * wx;
        dy += sqrt(2.0 * D * Gp * Dd.dt) * wy;
        dz += sqrt(2.0 * D * Gn * Dd.dt) * wz;
        nx = xi + dx;
        ny = yi + dy;
        nz = zi + dz;
        if (!(isfinite(nx) && isfinite(ny) && isfinite(nz))) {
            set_flag(flags, DISCOS_FLAG_NONFINITE);
            nx = xi;
            ny = yi;
            nz = zi;
        } else {
            nx = wrap_coord(nx, g.Lx);
            ny = wrap_coord(ny, g.Ly);
            nz = reflect_walls(nz, g.Lz);
        }
    } else {
        set_flag(flags, (isfinite(xi) && isfinite(yi) && isfinite(zi)) ? DISCOS_FLAG_OUT_OF_DOMAIN
                                                                     : DISCOS_FLAG_NONFINITE);
    }
    pos[i] = nx;
    pos[i + pstride] = ny;
    pos[i + 2 * pstride] = nz;
    q[i] = qi;
    id[i] = idi;
    sp[i] = sp_in;
}

int force_update_dry(Ctx* c, int n, const discos_params* p, uint64_t step, double* pos,
                     double* q, int* id, int* sp, hipStream_t s) {
    if (n <= 0) return DISCOS_OK;
    DryDev Dd;
    Dd.nsp = p->nspecies;
    Dd.kT = p->kT;
    Dd.eta = p->eta;
    Dd.dt = p->dt;
    Dd.radius = p->radius;
    Dd.coef = p->mob_coef;
    Dd.seed = p->seed;
    Dd.step = step;
    const int T = 128;
    force_update_dry_kernel<<<(n + T - 1) / T, T, 0, s>>>(
        c->gd, near_of(c, p), Dd, n, c->sxyzq, c->sid, c->ssp, c->bin_start,
        c->fp, c->n_max, pos, n, q, id, sp, c->flags);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
