// Particle-particle part of the step: the P3M near-field correction with wall images
// (eqs coulomb, fullElectro, LC and the image rule of Sec. II.B.1), the 9-3 wall
// force and the optional ion-ion LJ force (Sec. II.B.2), and the dry update
// (eq ions3, eq step2 with the tensor of eq diff1).  One lane per ion in cell-list
// order; neighbours come from the (2R+1)^2 rows of 2R+1 contiguous bins around the
// ion's bin, so consecutive lanes read overlapping, cache-resident candidates.
#include "kernels.h"

namespace discos {

struct NearDev {
    double psi, psi2, psi2g, inv4pieps, h, inv_h2, inv_hdr;
    double rsearch;  // search radius: psi, or the LJ range if larger
    const double* tab;
    int tablen;
    int R;  // search radius in bins
    double s_lo, s_hi;
    const int* map[2];  // per-column wall types (image sign of each source's column)
    int wall_on;
    double wsig, wxi, wcut;
    int lj_on;
    const double* ljs;
    const double* ljx;
    double ljf;
    int nsp;
};

static NearDev near_of_h(double h, const discos_params* p, int lb) {
    NearDev d;
    d.psi = p->psi;
    d.psi2 = p->psi * p->psi;
    d.psi2g = p->psi * p->psi * (1.0 + 1e-12);
    d.inv4pieps = 1.0 / (4.0 * M_PI * p->eps);
    d.h = h;
    d.inv_h2 = 1.0 / (h * h);
    d.inv_hdr = 1.0 / (h * p->p3m_dr);
    d.tab = p->p3m_table;
    d.tablen = p->p3m_len;
    double range = p->psi;
    if (p->lj_on) range = std::max(range, p->lj_range);
    d.rsearch = range;
    d.R = (int)std::ceil(range / ((double)(1 << lb) * h));
    d.s_lo = p->bc_type[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    d.s_hi = p->bc_type[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    d.map[0] = p->bc_type_map[0];
    d.map[1] = p->bc_type_map[1];
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

static NearDev near_of(const Ctx* c, const discos_params* p) { return near_of_h(c->grid.h, p, c->gd.lb); }

int near_radius_bins(const Ctx* c, const discos_params* p) { return near_of(c, p).R; }

int near_radius_bins_h(double h, const discos_params* p, int lb) { return near_of_h(h, p, lb).R; }

// 1/sqrt(r2) to full FP64 accuracy: hardware estimate plus two Newton steps.
__device__ __forceinline__ double inv_sqrt(double r2) {
    double y = __builtin_amdgcn_rsq(r2);
    y = y * (1.5 - 0.5 * r2 * y * y);
    y = y * (1.5 - 0.5 * r2 * y * y);
    return y;
}

// Pair force for 0 < r2 < psi^2: qq / (4 pi eps) [1/r^2 - g(r/h)/h^2] rhat.
__device__ __forceinline__ void es_pair_r2(double dx, double dy, double dz, double r2, double qq,
                                           const NearDev& P, double& fx, double& fy, double& fz) {
    const double inv_r = inv_sqrt(r2);
    const double r = r2 * inv_r;
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
    // dU/dr of 4 xi ((s/r)^12 - (s/r)^6), integer powers by multiplication
    const double sr = sig / r;
    const double sr2 = sr * sr;
    const double sr6 = sr2 * sr2 * sr2;
    const double du = 4.0 * xi * (-12.0 * sr6 * sr6 + 6.0 * sr6) / r;
    const double m = -du / r;
    fx += m * dx;
    fy += m * dy;
    fz += m * dz;
}

__device__ __forceinline__ double du93(double y, const NearDev& P) {
    if (!(y > 0.0 && y < P.wcut)) return 0.0;
    const double c93 = 1.5 * sqrt(3.0);
    const double sy = P.wsig / y;
    const double sy3 = sy * sy * sy;
    return c93 * P.wxi * (-9.0 * sy3 * sy3 * sy3 + 3.0 * sy3) / y;
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
    const double t52 = t5 * t5;
    return c[0] + c[1] / (c[2] + y) + c[3] / (t3 * t3 * t3) + c[5] / (t52 * t52 * t5);
}

__device__ __forceinline__ double dgamma_hat(double y, const double* c) {
    const double t1 = c[2] + y, t3 = c[4] + y, t5 = c[6] + y;
    const double t32 = t3 * t3, t52 = t5 * t5;
    return -c[1] / (t1 * t1) - 3.0 * c[3] / (t32 * t32) - 5.0 * c[5] / (t52 * t52 * t52);
}

// Update of one ion: the dry terms of eq ions3 / eq step2 (Euler-Maruyama, Ito) plus
// the wet displacement (wx0, wy0, wz0) = dt J(x*) v (zero in a dry step); returns the
// new position (wrapped in x, y, reflected at the walls).
__device__ __forceinline__ void dry_move(const GridDev& g, const DryDev& Dd, int spi, int idi,
                                         double xi, double yi, double zi, double Fx, double Fy,
                                         double Fz, double wx0, double wy0, double wz0,
                                         double& nx, double& ny, double& nz,
                                         int* __restrict__ flags) {
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
    nx = xi + (wx0 + dx);
    ny = yi + (wy0 + dy);
    nz = zi + (wz0 + dz);
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
}

// Update of every ion of the cell list from its complete force fp (grid, near field,
// wall, applied field) and, in a wet step, its velocity vw = J(x*) v, written to the
// caller's arrays in cell-list order.
// The update of ion gi of the cell list with complete force (Fx, Fy, Fz).
__device__ __forceinline__ void update_with_force(const GridDev& g, const DryDev& Dd, int gi,
                                                  double4 me, int sp_in, int idi, double Fx,
                                                  double Fy, double Fz, double wx0, double wy0,
                                                  double wz0, double* __restrict__ pos,
                                                  int64_t pstride, double* __restrict__ q,
                                                  int* __restrict__ id, int* __restrict__ sp,
                                                  int* __restrict__ flags) {
    const bool sp_ok = sp_in >= 0 && sp_in < Dd.nsp;
    if (!sp_ok) set_flag(flags, DISCOS_FLAG_BAD_SPECIES);
    const int spi = sp_ok ? sp_in : 0;
    double nx = me.x, ny = me.y, nz = me.z;
    if (pos_ok(g, me.x, me.y, me.z)) {
        dry_move(g, Dd, spi, idi, me.x, me.y, me.z, Fx, Fy, Fz, wx0, wy0, wz0, nx, ny, nz, flags);
    } else {
        set_flag(flags, (isfinite(me.x) && isfinite(me.y) && isfinite(me.z)) ? DISCOS_FLAG_OUT_OF_DOMAIN
                                                                          : DISCOS_FLAG_NONFINITE);
    }
    pos[gi] = nx;
    pos[gi + pstride] = ny;
    pos[gi + 2 * pstride] = nz;
    q[gi] = me.w;
    id[gi] = idi;
    sp[gi] = sp_in;
}

__device__ __forceinline__ void update_one(const GridDev& g, const DryDev& Dd, int gi,
                                           const double4* __restrict__ sxyzq,
                                           const int* __restrict__ sid, const int* __restrict__ ssp,
                                           const double* __restrict__ fp,
                                           const double* __restrict__ fp2, int64_t fstride,
                                           const double* __restrict__ vw, double* __restrict__ pos,
                                           int64_t pstride, double* __restrict__ q,
                                           int* __restrict__ id, int* __restrict__ sp,
                                           int* __restrict__ flags) {
    const double4 me = sxyzq[gi];
    const int sp_in = ssp[gi];
    const int idi = sid[gi];
    double wx0 = 0.0, wy0 = 0.0, wz0 = 0.0;
    if (vw) {
        wx0 = Dd.dt * vw[gi];
        wy0 = Dd.dt * vw[gi + fstride];
        wz0 = Dd.dt * vw[gi + 2 * fstride];
    }
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    if (pos_ok(g, me.x, me.y, me.z)) {
        Fx = fp[gi];
        Fy = fp[gi + fstride];
        Fz = fp[gi + 2 * fstride];
        if (fp2) {  // the grid force plus the near-field force computed apart
            Fx += fp2[gi];
            Fy += fp2[gi + fstride];
            Fz += fp2[gi + 2 * fstride];
        }
    }
    update_with_force(g, Dd, gi, me, sp_in, idi, Fx, Fy, Fz, wx0, wy0, wz0, pos, pstride, q, id, sp,
                      flags);
}

// Output of the force pass: out[o] += F (o = perm[i] if scatter), or with U.pos set, the
// dry step's update of ion i from its complete force out[i] + F (nothing reads the
// forces after a dry step), written to the caller's arrays in cell-list order.
struct FusedUpdate {
    DryDev Dd;
    const int* sid;
    double* pos;
    double* q;
    int* id;
    int* sp;
    int store;  // without an update: out[o] = F instead of out[o] += F
};

// ---- the near-field pass's padded cell list ----------------------------------------
// A copy of the cell list in which every search row of the pass is one contiguous run
// and every candidate already sits where the pair sees it.  Padded bins (px, py, pz),
// px in [0, nbx + 2R) (likewise y) and pz in [0, nbz + 2R + (nz odd)), x fastest:
//   - px - R and py - R are the real bins, periodic: the R bins on either side hold the
//     copies of the bins across the periodic seam, with x (y) shifted by the period;
//   - pz - R in [0, nbz) are the real slabs; the R slabs beyond each wall hold the
//     mirror images of the R slabs next to it (Sec. II.B.1): z -> -z below the lower
//     wall and z -> 2 Lz - z above the upper one, charge times the wall's image sign,
//     species -1 (the images carry no short-range force).
// Each real bin's ions keep their order in every copy, so the copy of the ion of rank k
// of a real bin is entry k of the padded bin.  Only first images are needed: a second
// reflection lies at least Lz >= 4 h away, beyond every cutoff the pass accepts.

// When nz is not a multiple of the bin edge B, the last real slab is th < B cells thick,
// and so is its mirror image above the upper wall: the image slabs there sit 2 (B - th)
// cells below where a slab grid continued through the wall would put them, and a window
// of R slabs above an ion reaches that much less far.  The upper side then gets
// ceil(2 (B - th) / B) image slabs more (one with two-cell bins and nz odd), and the
// pass searches as many slabs further up.
__host__ __device__ __forceinline__ int pad_top(const GridDev& g, int R) {
    if (g.lb == 1) return R + (g.nz & 1);
    const int B = 1 << g.lb, th = g.nz - ((g.nbz - 1) << g.lb);
    return R + (th >= B ? 0 : (2 * (B - th) + B - 1) / B);
}

// Real bin (channel-local) whose ions padded bin P holds, or -1 (a mirrored slab that
// does not exist in a channel thinner than the image layers).
__device__ __forceinline__ int pad_source(const GridDev& g, int R, int P) {
    const int PX = g.nbx + 2 * R, PY = g.nby + 2 * R;
    const int px = P % PX, py = (P / PX) % PY, pz = P / (PX * PY);
    const int bx = wrapi(px - R, g.nbx), by = wrapi(py - R, g.nby);
    int t = pz - R;
    if (t < 0)
        t = -t - 1;
    else if (t >= g.nbz)
        t = 2 * g.nbz - 1 - t;
    if (t < 0 || t >= g.nbz) return -1;
    return (t * g.nby + by) * g.nbx + bx;
}

int64_t near_list_bins(const GridDev& g, int R) {
    return (int64_t)(g.nbx + 2 * R) * (g.nby + 2 * R) * (g.nbz + R + pad_top(g, R));
}

// Copies per ion: at most two in x and two in y (2R + 1 <= nbx, nby, so no bin is within
// R of both seams), and in z the ion itself plus one image per wall within the image
// layers (both walls only when nbz < R + pad_top); sized for R up to 3.
int64_t near_list_entries(const GridDev& g, int64_t n) {
    return std::max<int64_t>(n, 1) * 4 * (g.nbz < 3 + pad_top(g, 3) ? 3 : 2);
}

__global__ void pad_count_kernel(GridDev g, int R, int64_t nb, const int* __restrict__ bin_start,
                                 int* __restrict__ count) {
    for (int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; P < nb;
         P += (int64_t)gridDim.x * blockDim.x) {
        const int s = pad_source(g, R, (int)P);
        count[P] = s < 0 ? 0 : bin_start[s + 1] - bin_start[s];
    }
}

// Batched: channels r = blockIdx.y, + gridDim.y, ..., whose padded bins are
// [pbin_off[r], pbin_off[r + 1]).
__global__ void pad_count_batch_kernel(const RepDev* __restrict__ reps, int nrep, int R,
                                       const int* __restrict__ pbin_off, const int* __restrict__ bin_start,
                                       int* __restrict__ count) {
    for (int r = blockIdx.y; r < nrep; r += gridDim.y) {
        const RepDev& Rp = reps[r];
        const int p0 = pbin_off[r], nb = pbin_off[r + 1] - p0;
        for (int P = blockIdx.x * blockDim.x + threadIdx.x; P < nb; P += gridDim.x * blockDim.x) {
            const int s = pad_source(Rp.g, R, P);
            count[p0 + P] = s < 0 ? 0 : bin_start[Rp.bin_off + s + 1] - bin_start[Rp.bin_off + s];
        }
    }
}

struct NlOut {
    double4* xyzq;
    float4* xyzf;
    int* sp;
    int64_t cap;
    int* flags;
};

// Every copy of sorted ion i (channel-local real bin b, rank k in it).  pstart: the
// channel's padded starts.  An ion outside the channel (flagged by the binning) still
// fills its slots, with coordinates that no distance test accepts.
__device__ __forceinline__ void pad_scatter_one(const GridDev& g, int R, int b, int k, double4 a,
                                                int spi, double s_lo, double s_hi,
                                                const int* const* map,
                                                const int* __restrict__ pstart, const NlOut& o) {
    const int PX = g.nbx + 2 * R, PY = g.nby + 2 * R;
    const int bx = b % g.nbx, by = (b / g.nbx) % g.nby, bz = b / (g.nbx * g.nby);
    const bool ok = pos_ok(g, a.x, a.y, a.z);
    if (ok && (map[0] || map[1])) {
        // a wall of mixed type: the image takes the type of the column below (above) the ion
        const int ci = min(max((int)floor(a.x * g.inv_h), 0), g.nx - 1);
        const int cj = min(max((int)floor(a.y * g.inv_h), 0), g.ny - 1);
        if (map[0]) s_lo = map[0][(size_t)cj * g.nx + ci] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
        if (map[1]) s_hi = map[1][(size_t)cj * g.nx + ci] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    }
    int pxs[2], pys[2], pzs[3], nzk = 1;
    double sxs[2], sys[2];
    int zkind[3];
    pxs[0] = bx + R;
    sxs[0] = 0.0;
    int ncx = 1;
    if (bx < R) { pxs[1] = bx + R + g.nbx; sxs[1] = g.Lx; ncx = 2; }
    else if (bx >= g.nbx - R) { pxs[1] = bx + R - g.nbx; sxs[1] = -g.Lx; ncx = 2; }
    pys[0] = by + R;
    sys[0] = 0.0;
    int ncy = 1;
    if (by < R) { pys[1] = by + R + g.nby; sys[1] = g.Ly; ncy = 2; }
    else if (by >= g.nby - R) { pys[1] = by + R - g.nby; sys[1] = -g.Ly; ncy = 2; }
    pzs[0] = bz + R;
    zkind[0] = 0;
    if (bz < R) { pzs[nzk] = R - 1 - bz; zkind[nzk++] = 1; }
    if (bz >= g.nbz - pad_top(g, R)) { pzs[nzk] = R + 2 * g.nbz - 1 - bz; zkind[nzk++] = 2; }
    const double bad = __builtin_nan("");
    for (int cz = 0; cz < nzk; ++cz) {
        const double zc = zkind[cz] == 0 ? a.z : (zkind[cz] == 1 ? -a.z : 2.0 * g.Lz - a.z);
        const double qc = zkind[cz] == 0 ? a.w : (zkind[cz] == 1 ? s_lo : s_hi) * a.w;
        const int spc = zkind[cz] == 0 ? spi : -1;
        for (int cy = 0; cy < ncy; ++cy)
            for (int cx = 0; cx < ncx; ++cx) {
                const int P = (pzs[cz] * PY + pys[cy]) * PX + pxs[cx];
                const int64_t d = (int64_t)pstart[P] + k;
                if (d >= o.cap) {
                    set_flag(o.flags, DISCOS_FLAG_CAPACITY);
                    continue;
                }
                const double xc = ok ? a.x + sxs[cx] : bad, yc = a.y + sys[cy];
                o.xyzq[d] = make_double4(xc, yc, zc, qc);
                o.xyzf[d] = make_float4((float)xc, (float)yc, (float)zc, 0.0f);
                o.sp[d] = spc;
            }
    }
}

// The cell-list bin of a sorted ion (x, y already reduced into [0, L]): the bin the
// binning gave it, for ions inside the channel.
__device__ __forceinline__ void sorted_bin(const GridDev& g, double x, double y, double z, int& bx,
                                           int& by, int& bz) {
    bx = min(max((int)floor(x * g.inv_h), 0), g.nx - 1) >> g.lb;
    by = min(max((int)floor(y * g.inv_h), 0), g.ny - 1) >> g.lb;
    bz = min(max((int)floor(z * g.inv_h), 0), g.nz - 1) >> g.lb;
}

__global__ void pad_scatter_kernel(GridDev g, int R, int n, double s_lo, double s_hi,
                                   const int* map_lo, const int* map_hi,
                                   const double4* __restrict__ sxyzq, const int* __restrict__ ssp,
                                   const int* __restrict__ perm, const int* __restrict__ ion_bin,
                                   const int* __restrict__ bin_start,
                                   const int* __restrict__ pstart, NlOut o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    g.lb = DISCOS_LB;  // a single channel's bins: a compile-time edge
    // the bin of an ion inside the channel follows from its sorted position (no dependent
    // loads through perm and ion_bin): the binning computed it from the same reduced
    // coordinates.  Others, and any slot outside that bin's range, take the bin the
    // binning recorded.
    const double4 a = sxyzq[i];
    int b = -1;
    if (pos_ok(g, a.x, a.y, a.z)) {
        int bx, by, bz;
        sorted_bin(g, a.x, a.y, a.z, bx, by, bz);
        b = (bz * g.nby + by) * g.nbx + bx;
        if (i < bin_start[b] || i >= bin_start[b + 1]) b = -1;
    }
    if (b < 0) b = ion_bin[perm[i]];
    if (i < bin_start[b] || i >= bin_start[b + 1]) {  // an inconsistent cell list
        set_flag(o.flags, DISCOS_FLAG_CAPACITY);
        return;
    }
    const int* map[2] = {map_lo, map_hi};
    pad_scatter_one(g, R, b, i - bin_start[b], a, ssp ? ssp[i] : 0, s_lo, s_hi, map, pstart, o);
}

__global__ void pad_scatter_batch_kernel(const RepDev* __restrict__ reps,
                                         const int* __restrict__ ion_rep, int R, int n,
                                         const double4* __restrict__ sxyzq,
                                         const int* __restrict__ ssp, const int* __restrict__ perm,
                                         const int* __restrict__ ion_bin,
                                         const int* __restrict__ bin_start,
                                         const int* __restrict__ pbin_off,
                                         const int* __restrict__ pstart, NlOut o) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = ion_rep[i];
    const RepDev& Rp = reps[r];
    const int b = ion_bin[perm[i]];  // batch-wide bin
    const int* const map[2] = {nullptr, nullptr};  // channels of a batch have uniform walls
    pad_scatter_one(Rp.g, R, b - Rp.bin_off, i - bin_start[b], sxyzq[i], ssp[i], Rp.s_lo, Rp.s_hi,
                    map, pstart + pbin_off[r], o);
}

// ---- the near-field pass ----------------------------------------------------------
// One lane per ion, consecutive ions of the cell list in consecutive lanes.  Each lane
// visits the 2R + 1 padded slabs around its ion (real slabs and, next to a wall, its
// image slabs):
//   1. the slab's 2R + 1 rows are cut to the search sphere (the slab and the row at
//      their nearest distance; in x the bins the sphere's chord reaches), and each
//      row's run of candidates goes to the lane's column of an LDS buffer;
//   2. one loop tests the slab's candidates in FP32 against the cutoff widened by a
//      bound of the FP32 error of the squared distance (coordinates below
//      2 Lmax, Lmax = max(Lx, Ly, 2 Lz), distances below the search radius: the margin
//      32 r_cut Lmax 2^-24), so the hits are a superset of the pairs, and appends every
//      hit (its padded index) to the lane's column of an LDS hit buffer;
//   3. as soon as one lane's buffer is full, every lane of the wavefront evaluates the
//      pairs in its own buffer (the exact FP64 cutoff, the P3M pair force, LJ) and
//      empties it; after the last slab the remaining buffers are evaluated.
// No neighbour list goes to memory, and the buffer size bounds nothing: denser systems
// only flush more often.  The slab and candidate loops have wavefront-uniform trip
// counts (a lane whose runs are exhausted idles), so a flush has every lane active.

#ifndef NF_THREADS
#define NF_THREADS 256  // four wavefronts per workgroup (they share the table)
#endif
#ifndef NF_HITS
#define NF_HITS 16      // hit buffer entries per lane (a multiple of NF_GROUP)
#endif
#ifndef NF_GROUP
#define NF_GROUP 1      // buffered pairs whose gathers are issued ahead together
#endif
#define NL_TAB 320

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

template <int R>
struct NfShared {
    int2 runs[2 * R + 2][NF_THREADS];  // a slab's runs, and one slot read past the last
    int hits[NF_HITS][NF_THREADS];
    double tab[NL_TAB];
};

// The padded list as the pass reads it.
struct NlView {
    const int* start;
    const double4* xyzq;
    const float4* xyzf;
    const int* sp;
};

// Pair forces of the m entries buffered in this lane's column (entry k at
// col[k * NF_THREADS]) on the ion at (xi, yi, zi) with charge qi, species spi.  The four
// gathers of a group of entries are issued together (a group's unused slots read the
// first entry's copy again).
__device__ __forceinline__ void nf_pairs(const int* col, int m, double xi, double yi, double zi,
                                         double qi, int spi, const NearDev& P, const NlView& L,
                                         double& fx, double& fy, double& fz) {
    const double r2lj = P.rsearch * P.rsearch * (1.0 + 1e-12);
    if (m <= 0) return;
    // group k + NF_GROUP's entries and gathers are in flight while group k is evaluated
    int e[NF_GROUP];
    double4 ob[NF_GROUP];
#pragma unroll
    for (int u = 0; u < NF_GROUP; ++u) e[u] = col[u * NF_THREADS];
#pragma unroll
    for (int u = 0; u < NF_GROUP; ++u) ob[u] = L.xyzq[u < m ? e[u] : e[0]];
    for (int k = 0; k < m; k += NF_GROUP) {
        const int m4 = min(NF_GROUP, m - k);
        const int kn = k + NF_GROUP < m ? k + NF_GROUP : k;
        int en[NF_GROUP];
        double4 obn[NF_GROUP];
#pragma unroll
        for (int u = 0; u < NF_GROUP; ++u) en[u] = col[(kn + u) * NF_THREADS];
#pragma unroll
        for (int u = 0; u < NF_GROUP; ++u) obn[u] = L.xyzq[kn + u < m ? en[u] : en[0]];
#pragma unroll
        for (int u = 0; u < NF_GROUP; ++u) {
            if (u >= m4) break;
            const double dx = xi - ob[u].x, dy = yi - ob[u].y, dz = zi - ob[u].z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            // the buffer is a superset (FP32 filter): the exact FP64 tests decide, and a
            // pair at zero separation has no direction and contributes nothing
            if (r2 < P.psi2 && r2 > 0.0) es_pair_r2(dx, dy, dz, r2, qi * ob[u].w, P, fx, fy, fz);
            if (P.lj_on && r2 < r2lj && r2 > 0.0) lj_pair(dx, dy, dz, spi, L.sp[e[u]], P, fx, fy, fz);
        }
#pragma unroll
        for (int u = 0; u < NF_GROUP; ++u) {
            e[u] = en[u];
            ob[u] = obn[u];
        }
    }
}

// Extent in z of padded slab t - R (t = pz - R, channel-local): a real slab, or the
// mirror image of one beyond a wall; empty (lo > hi) if that slab does not exist.
__device__ __forceinline__ void slab_extent(const GridDev& g, int t, double& lo, double& hi) {
    const double Bh = bin_edge(g);
    if (t >= 0 && t < g.nbz) {
        lo = t * Bh;
        hi = fmin((t + 1) * Bh, g.Lz);
    } else {
        const int s = t < 0 ? -t - 1 : 2 * g.nbz - 1 - t;
        if (s < 0 || s >= g.nbz) {
            lo = 1.0;
            hi = 0.0;
            return;
        }
        const double a = s * Bh, b = fmin((s + 1) * Bh, g.Lz);
        lo = t < 0 ? -b : 2.0 * g.Lz - b;
        hi = t < 0 ? -a : 2.0 * g.Lz - a;
    }
}

// Near-field, wall (and LJ) force of ion i of the cell list (x, y reduced into [0, L];
// real bin (bx, by, bz)) into (fx, fy, fz).  The ion's own entry among the candidates
// is a copy of its coordinates, so it passes the FP32 filter and is dropped by the
// exact test (zero separation), like any pair at zero separation.
template <int R>
__device__ __forceinline__ void nf_ion(const GridDev& g, const NearDev& P, int bx, int by, int bz,
                                       double4 me, int spi, const NlView& L,
                                       const int* __restrict__ pstart, NfShared<R>& sh,
                                       double& fx, double& fy, double& fz) {
    const int lane = threadIdx.x;
    const double xi = me.x, yi = me.y, zi = me.z, qi = me.w;
    const double Bh = bin_edge(g);
    const double inv_Bh = 1.0 / Bh;
    const double rs2 = P.rsearch * P.rsearch;
    const double r2cut = fmax(P.psi2, P.lj_on ? rs2 * (1.0 + 1e-12) : 0.0);
    const double Lmax = fmax(fmax(g.Lx, g.Ly), 2.0 * g.Lz);
    const double margin = 32.0 * sqrt(r2cut) * Lmax * 0x1.0p-24;
    const float xf = (float)xi, yf = (float)yi, zf = (float)zi;
    const int PX = g.nbx + 2 * R, PY = g.nby + 2 * R;
    int2* const rcol = &sh.runs[0][lane];
    int* const hcol = &sh.hits[0][lane];
    int cnt = 0;
    const int dz_hi = pad_top(g, R);  // more slabs up with offset upper image layers
#pragma unroll 1
    for (int dzb = -R; dzb <= dz_hi; ++dzb) {
        const int t = bz + dzb;
        const bool image = t < 0 || t >= g.nbz;
        double zb0, zb1;
        slab_extent(g, t, zb0, zb1);
        const double dzm = fmax(0.0, fmax(zb0 - zi, zi - zb1));
        // images carry only the electrostatic correction: their search radius is psi
        const double remz = (zb0 <= zb1) ? (image ? P.psi2 : rs2) - dzm * dzm : -1.0;
        const float cutf = (float)((image ? P.psi2 : r2cut) * (1.0 + 1e-5) + margin);
        // 1. the slab's runs, one per row: every row's bounds are computed and loaded
        // together (a row cut away loads a valid index and is dropped), then the
        // non-empty runs go to LDS
        int nr = 0;
        if (remz > 0.0) {
            const int slab = (t + R) * PY;
            int a0[2 * R + 1], a1[2 * R + 1];
            bool keep[2 * R + 1];
#pragma unroll
            for (int r = 0; r < 2 * R + 1; ++r) {
                const int dyb = r - R;
                const double yb0 = (by + dyb) * Bh;
                const double dym = fmax(0.0, fmax(yb0 - yi, yi - (yb0 + Bh)));
                const double rem = remz - dym * dym;
                // half chord of the search sphere in x; the FP32 root (within 2^-22
                // relative of the exact one) is widened so that the bin range can only grow
                const double wx = (double)__builtin_amdgcn_sqrtf((float)fmax(rem, 0.0)) *
                                      (1.0 + 0x1.0p-18) + 0x1.0p-20 * Bh;
                const int bxl = max(bx - R, (int)floor((xi - wx) * inv_Bh));
                const int bxh = min(bx + R, (int)floor((xi + wx) * inv_Bh));
                keep[r] = rem > 0.0 && bxl <= bxh;
                const int row = (slab + by + dyb + R) * PX + R;
                a0[r] = keep[r] ? row + bxl : row;
                a1[r] = keep[r] ? row + bxh + 1 : row;
            }
            int j0[2 * R + 1], j1[2 * R + 1];
#pragma unroll
            for (int r = 0; r < 2 * R + 1; ++r) {
                j0[r] = pstart[a0[r]];
                j1[r] = pstart[a1[r]];
            }
#pragma unroll
            for (int r = 0; r < 2 * R + 1; ++r)
                if (keep[r] && j0[r] < j1[r]) rcol[(nr++) * NF_THREADS] = make_int2(j0[r], j1[r]);
        }
        // 2. their candidates in one loop without branches: each iteration first steps
        // to the next candidate (the next run's bounds were read from LDS ahead of time)
        // and issues its load, then tests the current one, whose coordinates arrived
        // meanwhile, and writes it to the hit buffer's next slot (kept only on a hit).
        int j = 0, je = 0, k = 0;
        if (nr > 0) {
            const int2 u = rcol[0];
            j = u.x;
            je = u.y;
            k = 1;
        }
        int2 un = rcol[k * NF_THREADS];  // the run after the current one (if k < nr)
        float4 o = L.xyzf[j < je ? j : 0];
        for (;;) {
            const bool act = j < je;
            if (!wave_any(act)) break;
            const bool sw = j + 1 >= je && k < nr;
            const int jn = act ? (sw ? un.x : j + 1) : je;
            const int jen = sw ? un.y : je;
            k += sw ? 1 : 0;
            const float4 on = L.xyzf[jn < jen ? jn : 0];
            if (sw) un = rcol[k * NF_THREADS];
            const float dx = xf - o.x, dy = yf - o.y, dz = zf - o.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            // a zero FP32 distance may be a distinct (coincident in FP32) pair
            const bool hit = act && r2 < cutf;
            hcol[cnt * NF_THREADS] = j;
            cnt += hit ? 1 : 0;
            j = jn;
            je = jen;
            o = on;
            // 3. a full buffer anywhere: every lane evaluates and empties its own
            if (wave_any(cnt == NF_HITS)) {
                nf_pairs(hcol, cnt, xi, yi, zi, qi, spi, P, L, fx, fy, fz);
                cnt = 0;
            }
        }
    }
    nf_pairs(hcol, cnt, xi, yi, zi, qi, spi, P, L, fx, fy, fz);
    if (P.wall_on) fz += -du93(zi, P) + du93(g.Lz - zi, P);
}


// Order of the pass's blocks within each XCD.  Block L covers ions [L NF_THREADS, ...) of
// the cell list, whose bins run z-slab by z-slab, so the blocks form about T = nbz rows
// (slabs) of W = ceil(nb / T) blocks, each row running through the slab's y rows.  The
// order enumerates 8 column bands of that matrix (y bands of the channel) one after the
// other, and each band slab by slab; xcd_block then hands XCD x the x-th eighth of this
// order, about one band.  The blocks an XCD has in flight (a few hundred) then span many
// slabs of one band rather than a few whole slabs, so the candidate slabs the pass reads
// stay in that XCD's L2 while the band sweeps through them.  A bijection on [0, nb).
__host__ __device__ inline int band_block(int p, int nb, int T) {
    const int W = (nb + T - 1) / T;
    T = (nb + W - 1) / W;  // rows actually used: the last one holds 1 to W blocks
    if (T < 2 || W < DISCOS_NXCD) return p;
    const int Wb = (W + DISCOS_NXCD - 1) / DISCOS_NXCD;  // band width in blocks
    const int last = nb - (T - 1) * W;                   // blocks in the last slab, 1..W
    for (int b = 0; b < DISCOS_NXCD; ++b) {
        const int c0 = b * Wb;
        const int wb = max(0, min(Wb, W - c0));
        const int tail = max(0, min(wb, last - c0));  // the band's blocks in the last slab
        const int cnt = (T - 1) * wb + tail;
        if (p < cnt) {
            if (p < (T - 1) * wb) return (p / wb) * W + c0 + p % wb;
            return (T - 1) * W + c0 + (p - (T - 1) * wb);
        }
        p -= cnt;
    }
    return p;  // not reached: the bands' counts sum to nb
}

// The pass over every ion of a context (BATCH = false: out[o] += F with o = perm[i] if
// scatter, else i; or with U.pos set, the dry step's update from the complete force
// out[i] + F) or of a batch (BATCH = true: ion i belongs to channel ion_rep[i], whose
// grid, bins and padded bins it uses; out[i] += F).
#ifndef NF_MINW
#define NF_MINW 5  // waves per SIMD the register allocation is held to
#endif
template <int R, bool BATCH>
__global__ void __launch_bounds__(NF_THREADS, NF_MINW)
near_field_kernel(GridDev g0, const RepDev* __restrict__ reps, const int* __restrict__ ion_rep,
                  const int* __restrict__ pbin_off, NearDev P, int n,
                  const double4* __restrict__ sxyzq, const int* __restrict__ ssp,
                  NlView L, const int* __restrict__ perm,
                  double* __restrict__ out, int64_t stride, int scatter, int* __restrict__ flags,
                  FusedUpdate U) {
    __shared__ NfShared<R> sh;
    const int nt = min(P.tablen, NL_TAB);
    for (int k = threadIdx.x; k < nt; k += NF_THREADS) sh.tab[k] = P.tab[k];
    __syncthreads();
    P.tab = sh.tab;
    const int i = (BATCH ? (int)blockIdx.x
                         : band_block(xcd_block(blockIdx.x, gridDim.x), gridDim.x, g0.nbz)) *
                      NF_THREADS +
                  (int)threadIdx.x;
    if (i >= n) return;
    GridDev g = g0;
    if (!BATCH) g.lb = DISCOS_LB;  // a single channel's bins: a compile-time edge
    const int* pstart = L.start;
    if (BATCH) {
        const int r = ion_rep[i];
        g = reps[r].g;
        pstart += pbin_off[r];
    }
    const double4 me = sxyzq[i];
    if (!pos_ok(g, me.x, me.y, me.z)) {
        if (!BATCH && U.pos)
            update_with_force(g, U.Dd, i, me, ssp[i], U.sid[i], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, U.pos, n,
                              U.q, U.id, U.sp, flags);
        return;
    }
    int spi = 0;
    if (P.lj_on) {
        spi = ssp[i];
        if (spi < 0 || spi >= max(P.nsp, 1)) set_flag(flags, DISCOS_FLAG_BAD_SPECIES);
    }
    int bx, by, bz;
    sorted_bin(g, me.x, me.y, me.z, bx, by, bz);
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    nf_ion<R>(g, P, bx, by, bz, me, spi, L, pstart, sh, Fx, Fy, Fz);
    if (BATCH) {
        out[i] += Fx;
        out[i + stride] += Fy;
        out[i + 2 * stride] += Fz;
        return;
    }
    if (U.pos) {
        update_with_force(g, U.Dd, i, me, ssp[i], U.sid[i], out[i] + Fx, out[i + stride] + Fy,
                          out[i + 2 * stride] + Fz, 0.0, 0.0, 0.0, U.pos, n, U.q, U.id, U.sp, flags);
        return;
    }
    const int o = scatter ? perm[i] : i;
    if (U.store) {
        out[o] = Fx;
        out[o + stride] = Fy;
        out[o + 2 * stride] = Fz;
        return;
    }
    out[o] += Fx;
    out[o + stride] += Fy;
    out[o + 2 * stride] += Fz;
}

// The pass for search radii of 1 to 3 bins (larger radii are rejected up front).
static int launch_near(const NearDev& P, int n, hipStream_t s, const GridDev& g,
                       const RepDev* reps, const int* ion_rep, const int* pbin_off,
                       const double4* sxyzq, const int* ssp, const NlView& L,
                       const int* perm, double* out, int64_t stride, int scatter, int* flags,
                       const FusedUpdate& U) {
    if (P.R < 1 || P.R > 3) return DISCOS_E_ARG;
    const int nb = (n + NF_THREADS - 1) / NF_THREADS;
#define NF_LAUNCH(RR)                                                                         \
    if (reps)                                                                                 \
        near_field_kernel<RR, true><<<nb, NF_THREADS, 0, s>>>(g, reps, ion_rep, pbin_off, P, n, \
                                                              sxyzq, ssp, L, perm,  \
                                                              out, stride, scatter, flags, U); \
    else                                                                                      \
        near_field_kernel<RR, false><<<nb, NF_THREADS, 0, s>>>(g, reps, ion_rep, pbin_off, P, n, \
                                                               sxyzq, ssp, L, perm, \
                                                               out, stride, scatter, flags, U);
    if (P.R == 1) {
        NF_LAUNCH(1)
    } else if (P.R == 2) {
        NF_LAUNCH(2)
    } else {
        NF_LAUNCH(3)
    }
#undef NF_LAUNCH
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

// The padded list of a context's cell list for search radius R.
static int build_near_list(Ctx* c, int n, int R, double s_lo, double s_hi, const int* const* map,
                           hipStream_t s) {
    const GridDev& g = c->gd;
    const int64_t nb = near_list_bins(g, R);
    if (nb > c->nl.bins_cap) return DISCOS_E_ARG;
    pad_count_kernel<<<(int)std::min<int64_t>((nb + 255) / 256, 4096), 256, 0, s>>>(
        g, R, nb, c->bin_start, c->nl.count);
    scan_counts(c->nl.count, nb, c->nl.tmp, c->nl.start, s);
    const NlOut o{c->nl.xyzq, c->nl.xyzf, c->nl.sp, c->nl.cap, c->flags};
    pad_scatter_kernel<<<(n + 255) / 256, 256, 0, s>>>(g, R, n, s_lo, s_hi, map[0], map[1], c->sxyzq,
                                                       c->ssp, c->perm,
                                                       c->ion_bin, c->bin_start, c->nl.start, o);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

static DryDev dry_of(const discos_params* p, uint64_t step) {
    DryDev Dd;
    Dd.nsp = p->nspecies;
    Dd.kT = p->kT;
    Dd.eta = p->eta;
    Dd.dt = p->dt;
    Dd.radius = p->radius;
    Dd.coef = p->mob_coef;
    Dd.seed = p->seed;
    Dd.step = step;
    return Dd;
}

int near_field_sorted(Ctx* c, int n, const discos_params* p, double* out, int64_t out_stride,
                      int scatter_to_caller, hipStream_t s, int mark, const DryStepOut* upd,
                      bool store) {
    if (n <= 0) return DISCOS_OK;
    const NearDev P = near_of(c, p);
    if (P.R < 1 || P.R > 3) return DISCOS_E_ARG;
    int rc = build_near_list(c, n, P.R, P.s_lo, P.s_hi, P.map, s);
    if (rc) return rc;
    if (mark >= 0) stage_mark(c, mark, s);
    FusedUpdate U{};
    U.store = store ? 1 : 0;
    if (upd) {
        U.Dd = dry_of(p, upd->step);
        U.sid = c->sid;
        U.pos = upd->pos;
        U.q = upd->q;
        U.id = upd->id;
        U.sp = upd->sp;
    }
    const NlView L{c->nl.start, c->nl.xyzq, c->nl.xyzf, c->nl.sp};
    rc = launch_near(P, n, s, c->gd, nullptr, nullptr, nullptr, c->sxyzq, c->ssp, L,
                     c->perm, out, out_stride, scatter_to_caller, c->flags, U);
    if (mark >= 0) stage_mark(c, mark + 1, s);
    return rc;
}

__global__ void dry_update_kernel(GridDev g, DryDev Dd, int n, const double4* __restrict__ sxyzq,
                                  const int* __restrict__ sid, const int* __restrict__ ssp,
                                  const double* __restrict__ fp, const double* __restrict__ fp2,
                                  int64_t fstride,
                                  const double* __restrict__ vw,
                                  double* __restrict__ pos, int64_t pstride, double* __restrict__ q,
                                  int* __restrict__ id, int* __restrict__ sp,
                                  int* __restrict__ flags) {
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= n) return;
    update_one(g, Dd, gi, sxyzq, sid, ssp, fp, fp2, fstride, vw, pos, pstride, q, id, sp, flags);
}

// Batched: each ion's channel supplies its grid, noise key and mobility fit; the step
// index is read from device memory (it advances with captured-graph replays).
__global__ void dry_update_batch_kernel(const RepDev* __restrict__ reps,
                                        const int* __restrict__ ion_rep, DryDev Dd,
                                        const uint64_t* __restrict__ step, int n,
                                        const double4* __restrict__ sxyzq,
                                        const int* __restrict__ sid, const int* __restrict__ ssp,
                                        const double* __restrict__ fp, double* __restrict__ pos,
                                        double* __restrict__ q, int* __restrict__ id,
                                        int* __restrict__ sp, int* __restrict__ flags) {
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= n) return;
    const RepDev& R = reps[ion_rep[gi]];
    Dd.seed = R.seed;
    Dd.coef = R.coef;
    Dd.step = *step;
    update_one(R.g, Dd, gi, sxyzq, sid, ssp, fp, nullptr, n, nullptr, pos, n, q, id, sp, flags);
}

__global__ void step_advance_kernel(uint64_t* step) { *step += 1; }
__global__ void step_set_kernel(uint64_t* step, uint64_t v) { *step = v; }

int batch_near(Batch* b, hipStream_t s) {
    const int n = (int)b->n_tot;
    if (n == 0) return DISCOS_OK;
    const NearDev P = near_of_h(b->h, &b->p, b->cfg.lb);
    if (P.R < 1 || P.R > 3) return DISCOS_E_ARG;
    const int nrep = (int)b->reps.size();
    pad_count_batch_kernel<<<dim3(b->pbin_xblocks, std::min(nrep, 65535)), 256, 0, s>>>(
        b->reps_d, nrep, P.R, b->pbin_off, b->bin_start, b->nl.count);
    scan_counts(b->nl.count, b->pbins_tot, b->nl.tmp, b->nl.start, s);
    const NlOut o{b->nl.xyzq, b->nl.xyzf, b->nl.sp, b->nl.cap, b->flags};
    const int T = b->cfg.ion_block;
    pad_scatter_batch_kernel<<<(n + T - 1) / T, T, 0, s>>>(b->reps_d, b->ion_rep, P.R, n, b->sxyzq,
                                                         b->ssp, b->perm, b->ion_bin, b->bin_start,
                                                         b->pbin_off, b->nl.start, o);
    const NlView L{b->nl.start, b->nl.xyzq, b->nl.xyzf, b->nl.sp};
    GridDev g{};
    return launch_near(P, n, s, g, b->reps_d, b->ion_rep, b->pbin_off, b->sxyzq, b->ssp, L,
                       nullptr, b->fp, n, 0, b->flags, FusedUpdate{});
}

int batch_update(Batch* b, double* pos, double* q, int* id, int* sp, hipStream_t s) {
    const int n = (int)b->n_tot;
    if (n == 0) return DISCOS_OK;
    DryDev Dd;
    Dd.nsp = b->p.nspecies;
    Dd.kT = b->p.kT;
    Dd.eta = b->p.eta;
    Dd.dt = b->p.dt;
    Dd.radius = b->p.radius;
    Dd.coef = nullptr;
    Dd.seed = 0;
    Dd.step = 0;
    const int T = b->cfg.ion_block;
    dry_update_batch_kernel<<<(n + T - 1) / T, T, 0, s>>>(b->reps_d, b->ion_rep, Dd, b->step_d, n,
                                                          b->sxyzq, b->sid, b->ssp, b->fp, pos, q, id,
                                                          sp, b->flags);
    step_advance_kernel<<<1, 1, 0, s>>>(b->step_d);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int batch_set_step(Batch* b, uint64_t v, hipStream_t s) {
    step_set_kernel<<<1, 1, 0, s>>>(b->step_d, v);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int update_sorted(Ctx* c, int n, const discos_params* p, uint64_t step, const double* vwet,
                  double* pos, double* q, int* id, int* sp, hipStream_t s, const double* fp2) {
    if (n <= 0) return DISCOS_OK;
    const DryDev Dd = dry_of(p, step);
    dry_update_kernel<<<(n + 255) / 256, 256, 0, s>>>(c->gd, Dd, n, c->sxyzq, c->sid, c->ssp, c->fp,
                                                      fp2, c->n_max, vwet, pos, n, q, id, sp,
                                                      c->flags);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
