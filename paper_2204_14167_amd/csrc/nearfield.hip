// Particle-particle part of the step: the P3M near-field correction with wall images
// (eqs coulomb, fullElectro, LC and the image rule of Sec. II.B.1), the 9-3 wall
// force and the optional ion-ion LJ force (Sec. II.B.2), and the dry update
// (eq ions3, eq step2 with the tensor of eq diff1).  One thread per ion in cell-list
// order; neighbours come from the (2R+1)^2 rows of 2R+1 contiguous bins around the
// ion's bin, so consecutive threads read overlapping, cache-resident neighbour lists.
#include "kernels.h"

namespace discos {

#define NL_CAP_DEFAULT 64  // list entries per ion of a single context

struct NearDev {
    double psi, psi2, psi2g, inv4pieps, h, inv_h2, inv_hdr;
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
    int cap;  // list entries per ion (a multiple of 4); longer lists take the cache-read path
};

static NearDev near_of_h(double h, const discos_params* p) {
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
    d.R = (int)std::ceil(range / (DISCOS_BIN * h));
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
    d.cap = NL_CAP_DEFAULT;
    return d;
}

static NearDev near_of(const Ctx* c, const discos_params* p) { return near_of_h(c->grid.h, p); }

int near_radius_bins(const Ctx* c, const discos_params* p) { return near_of(c, p).R; }

// List capacity for ion densities up to rho_max (ions per unit volume): the mean number
// of candidates inside the search sphere (wall images replace the part of the sphere
// beyond a wall, so the sphere bounds them), 25 % more for the FP32 margin and bin
// shapes, plus six standard deviations; at least the single-context capacity.
int near_list_capacity(double h, const discos_params* p, double rho_max) {
    const double r = near_of_h(h, p).rsearch;
    const double mean = 1.25 * (4.0 / 3.0) * M_PI * r * r * r * rho_max;
    const int cap = (int)std::ceil(mean + 6.0 * std::sqrt(mean) + 16.0);
    return std::max(NL_CAP_DEFAULT, (cap + 3) & ~3);
}
int near_radius_bins_h(double h, const discos_params* p) { return near_of_h(h, p).R; }

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

// F^C - F^P for one pair (or ion-image pair) at separation d, charge product qq.
// A pair at zero separation has no direction and contributes nothing.
__device__ __forceinline__ void es_pair(double dx, double dy, double dz, double qq,
                                        const NearDev& P, double& fx, double& fy, double& fz) {
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < P.psi2) || !(r2 > 0.0)) return;
    es_pair_r2(dx, dy, dz, r2, qq, P, fx, fy, fz);
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

// ---- global-memory path (one thread per ion, candidates read through the caches) ----
// Used only for blocks whose neighbourhood does not fit the LDS stage (very dense
// clusters); the staged path below is the normal one.
__device__ void near_force_global(int i, double4 me, int spi, const double4* __restrict__ sxyzq,
                                  const int* __restrict__ ssp, const int* __restrict__ bin_start,
                                  const GridDev& g, const NearDev& P, double& Fx, double& Fy,
                                  double& Fz) {
    const double xi = me.x, yi = me.y, zi = me.z, qi = me.w;
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
        for (int cz = zlo; cz <= zhi; ++cz)
            for (int dyb = -P.R; dyb <= P.R; ++dyb) {
                const int cyu = by + dyb;
                const int cy = cyu < 0 ? cyu + g.nby : (cyu >= g.nby ? cyu - g.nby : cyu);
                const double ys = yi - (cyu < 0 ? -g.Ly : (cyu >= g.nby ? g.Ly : 0.0));
                const int row = (cz * g.nby + cy) * g.nbx;
                for (int dxb = -P.R; dxb <= P.R; ++dxb) {
                    const int cxu = bx + dxb;
                    const int cx = cxu < 0 ? cxu + g.nbx : (cxu >= g.nbx ? cxu - g.nbx : cxu);
                    const double xs = xi - (cxu < 0 ? -g.Lx : (cxu >= g.nbx ? g.Lx : 0.0));
                    const int j0 = bin_start[row + cx], j1 = bin_start[row + cx + 1];
                    for (int j = j0; j < j1; ++j) {
                        const double4 o = sxyzq[j];
                        const double dx = xs - o.x, dy = ys - o.y;
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
    Fx = fx;
    Fy = fy;
    Fz = fz;
}

// ---- neighbour list + force pass -------------------------------------------------
// Pass 1 (one thread per ion of the cell list): visit the rows of bins around the ion
// (a row is skipped when its slab is farther than the search radius and cut to the
// x-bins that can reach the sphere; periodic copies and wall images carry a shift /
// mode code), test each candidate's distance, and append the hits to the ion's list.
// Pass 2 (one thread per ion) evaluates the pair forces of its list.  The
// distance test, whose trip count differs between lanes, is thereby separated from the
// pair arithmetic, which then runs only on pairs inside the cutoff.  Lists are written
// and read in chunks of four entries; chunk c of ion i sits at [c * n + i], so the
// chunk reads of a wavefront are contiguous.
#define NL_TAB 320

__device__ __forceinline__ double shift_of(int code, double L) {
    return code == 1 ? -L : (code == 2 ? L : 0.0);
}

// Runs of candidate bins of one slab (one z-row of bins, or one image layer), at most
// two per y-row: 2R + 1 <= nbx, so a row of 2R + 1 bins crosses the periodic seam at
// most once.  Each thread keeps its slab's runs in its own column of the block's LDS
// buffer (entry = first sorted index | shift and mode code, end index).
#define NL_SLAB_RUNS(R) (2 * (2 * (R) + 1))

// A run entry decoded: its candidate range, code bits, and the ion's x and y against
// the candidates' periodic copy.
struct NlRun {
    int j, e, code;
    float xs, ys;
};

__device__ __forceinline__ NlRun nl_run(int2 r, float xf0, float xf1, float xf2, float yf0,
                                        float yf1, float yf2) {
    NlRun u;
    u.j = r.x & 0x3FFFFFF;
    u.code = r.x & ~0x3FFFFFF;
    u.e = r.y;
    const int xc = (r.x >> 26) & 3, yc = (r.x >> 28) & 3;
    u.xs = xc == 0 ? xf0 : (xc == 1 ? xf1 : xf2);
    u.ys = yc == 0 ? yf0 : (yc == 1 ? yf1 : yf2);
    return u;
}

template <int R>
__device__ __forceinline__ void near_list_one(const GridDev& g, const NearDev& P, int i, int n,
                                              const double4* __restrict__ sxyzq,
                                              const float4* __restrict__ sxyzf,
                                              const int* __restrict__ bin_start,
                                              int* __restrict__ list, int* __restrict__ count,
                                              int2* __restrict__ buf, int bstride) {
    const double4 me = sxyzq[i];
    const double xi = me.x, yi = me.y, zi = me.z;
    if (!pos_ok(g, xi, yi, zi)) {
        count[i] = 0;
        return;
    }
    const double Bh = DISCOS_BIN * g.h;
    const double inv_Bh = 1.0 / Bh;
    const double rs2 = P.rsearch * P.rsearch;
    const double r2cut = fmax(P.psi2, P.lj_on ? rs2 * (1.0 + 1e-12) : 0.0);
    int bx, by, bz;
    bin_of(g, xi, yi, zi, bx, by, bz);
    // Candidates are filtered in FP32 against the cutoff widened by a margin that bounds
    // the FP32 error of the squared distance (coordinates up to Lmax, distances up to
    // the search radius): the lists are a superset of the pairs inside the cutoff, and
    // the force pass applies the exact FP64 test.
    const double Lmax = fmax(fmax(g.Lx, g.Ly), 2.0 * g.Lz);
    const double margin = 32.0 * sqrt(r2cut) * Lmax * 0x1.0p-24;
    // the ion's coordinates against a candidate's periodic copy, by shift code 0, 1, 2
    float xf0 = (float)xi, xf1 = (float)(xi + g.Lx), xf2 = (float)(xi - g.Lx);
    float yf0 = (float)yi, yf1 = (float)(yi + g.Ly), yf2 = (float)(yi - g.Ly);
    // opaque to the optimiser: otherwise it folds the per-run choice of these six values
    // back into an FP64 add and conversion inside the candidate loop
    asm("" : "+v"(xf0), "+v"(xf1), "+v"(xf2), "+v"(yf0), "+v"(yf1), "+v"(yf2));
    // chunk c of ion i at [c * n + i]; the last four hits are kept in h0..h3 (oldest first)
    int4* const chunks = reinterpret_cast<int4*>(list) + i;
    int nh = 0, h0 = 0, h1 = 0, h2 = 0, h3 = 0;
    for (int mode = 0; mode < 3; ++mode) {
        int zlo, zhi;
        if (mode == 0) {
            zlo = max(bz - R, 0);
            zhi = min(bz + R, g.nbz - 1);
        } else if (mode == 1) {
            if (!(zi < P.psi)) continue;
            zlo = 0;
            zhi = min(g.nbz - 1, (int)floor(P.psi * g.inv_h) / DISCOS_BIN);
        } else {
            if (!(zi > g.Lz - P.psi)) continue;
            zlo = max(0, (int)floor((g.Lz - P.psi) * g.inv_h) / DISCOS_BIN);
            zhi = g.nbz - 1;
        }
        const double r2m = mode == 0 ? rs2 : P.psi2;
        const double cut = mode == 0 ? r2cut : P.psi2;
        const float zsf = mode == 0 ? 1.0f : -1.0f;
        const float zef = (float)(mode == 2 ? zi - 2.0 * g.Lz : zi);
        const float cutf = (float)(cut * (1.0 + 1e-5) + margin);
        const int self = mode == 0 ? i : -1;  // the ion itself is excluded by index
        const int mcode = mode << 30;
        for (int cz = zlo; cz <= zhi; ++cz) {
            const double zb0 = cz * Bh, zb1 = fmin((cz + 1) * Bh, g.Lz);
            const double dzm = mode == 0 ? fmax(0.0, fmax(zb0 - zi, zi - zb1))
                                         : (mode == 1 ? zi + zb0 : (2.0 * g.Lz - zb1) - zi);
            const double remz = r2m - dzm * dzm;
            if (!(remz > 0.0)) continue;
            // 1. the slab's non-empty runs
            int nr = 0;
#pragma unroll 1
            for (int dyb = -R; dyb <= R; ++dyb) {
                const int cyu = by + dyb;
                const double yb0 = cyu * Bh;
                const double dym = fmax(0.0, fmax(yb0 - yi, yi - (yb0 + Bh)));
                const double rem = remz - dym * dym;
                if (!(rem > 0.0)) continue;
                // half chord of the search sphere in x; the FP32 root (within 2^-22
                // relative of the exact one) is widened so that the bin range can only grow
                const double wx =
                    (double)__builtin_amdgcn_sqrtf((float)rem) * (1.0 + 0x1.0p-18) + 0x1.0p-20 * Bh;
                const int bxl = max(bx - R, (int)floor((xi - wx) * inv_Bh));
                const int bxh = min(bx + R, (int)floor((xi + wx) * inv_Bh));
                if (bxl > bxh) continue;
                const int cy = cyu < 0 ? cyu + g.nby : (cyu >= g.nby ? cyu - g.nby : cyu);
                const int ycode = (cyu < 0 ? 1 : (cyu >= g.nby ? 2 : 0)) << 28;
                const int row = (cz * g.nby + cy) * g.nbx;
                // first run: up to the seam (or the whole range)
                const int e1 = bxl < 0 ? min(bxh, -1) : (bxl < g.nbx ? min(bxh, g.nbx - 1) : bxh);
                const int cx1 = bxl < 0 ? bxl + g.nbx : (bxl >= g.nbx ? bxl - g.nbx : bxl);
                const int xc1 = bxl < 0 ? 1 : (bxl >= g.nbx ? 2 : 0);
                const int j0 = bin_start[row + cx1], j1 = bin_start[row + cx1 + (e1 - bxl) + 1];
                // second run: past the seam
                const bool two = e1 < bxh;
                const int b2 = e1 + 1;
                const int cx2 = b2 >= g.nbx ? b2 - g.nbx : b2;
                const int xc2 = b2 >= g.nbx ? 2 : 0;
                const int k0 = two ? bin_start[row + cx2] : 0;
                const int k1 = two ? bin_start[row + cx2 + (bxh - b2) + 1] : 0;
                if (j0 < j1) buf[(nr++) * bstride] = make_int2(j0 | (xc1 << 26) | ycode | mcode, j1);
                if (k0 < k1) buf[(nr++) * bstride] = make_int2(k0 | (xc2 << 26) | ycode | mcode, k1);
            }
            // 2. their candidates in one loop: a lane's trip count is its slab total.  The
            // next candidate (and, at a run's end, the next run from LDS) is found while
            // the current one's coordinates are in flight.
            const int2* rp = buf;
            const int2* const rend = buf + nr * bstride;
            int j = 0, je = 0, code = 0;
            float xs = 0.0f, ys = 0.0f;
            if (rp < rend) {
                const NlRun u = nl_run(*rp, xf0, xf1, xf2, yf0, yf1, yf2);
                j = u.j;
                je = u.e;
                code = u.code;
                xs = u.xs;
                ys = u.ys;
                rp += bstride;
            }
            while (j < je) {
                const float4 o = sxyzf[j];
                int jn = j + 1, jen = je, coden = code;
                float xsn = xs, ysn = ys;
                if (jn >= je && rp < rend) {
                    const NlRun u = nl_run(*rp, xf0, xf1, xf2, yf0, yf1, yf2);
                    jn = u.j;
                    jen = u.e;
                    coden = u.code;
                    xsn = u.xs;
                    ysn = u.ys;
                    rp += bstride;
                }
                const float dx = xs - o.x;
                const float dy = ys - o.y;
                const float dz = zef - zsf * o.z;
                const float r2 = dx * dx + dy * dy + dz * dz;
                // a zero FP32 distance may be a distinct (coincident in FP32) pair
                if (r2 < cutf && j != self) {
                    h0 = h1;
                    h1 = h2;
                    h2 = h3;
                    h3 = j | code;
                    ++nh;
                    if ((nh & 3) == 0 && nh <= P.cap)
                        chunks[(size_t)((nh >> 2) - 1) * n] = make_int4(h0, h1, h2, h3);
                }
                j = jn;
                je = jen;
                code = coden;
                xs = xsn;
                ys = ysn;
            }
        }
    }
    // the incomplete last chunk: its m = nh mod 4 hits are the newest m of h0..h3
    const int m = nh & 3;
    if (m && nh <= P.cap)
        chunks[(size_t)(nh >> 2) * n] =
            m == 1 ? make_int4(h3, 0, 0, 0) : (m == 2 ? make_int4(h2, h3, 0, 0) : make_int4(h1, h2, h3, 0));
    count[i] = nh;
}

template <int R>
__global__ void __launch_bounds__(256)
near_list_kernel(GridDev g, NearDev P, int n, const double4* __restrict__ sxyzq,
                 const float4* __restrict__ sxyzf,
                 const int* __restrict__ bin_start, int* __restrict__ list,
                 int* __restrict__ count) {
    extern __shared__ int2 nl_buf[];
    const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    near_list_one<R>(g, P, i, n, sxyzq, sxyzf, bin_start, list, count, nl_buf + threadIdx.x,
                     blockDim.x);
}

// Batched: ion i (cell-list order) belongs to channel ion_rep[i]; its bins start at the
// channel's bin offset, and its list entries are batch-wide sorted indices.
template <int R>
__global__ void __launch_bounds__(256)
near_list_batch_kernel(const RepDev* __restrict__ reps, const int* __restrict__ ion_rep,
                       NearDev P, int n, const double4* __restrict__ sxyzq,
                       const float4* __restrict__ sxyzf,
                       const int* __restrict__ bin_start, int* __restrict__ list,
                       int* __restrict__ count) {
    extern __shared__ int2 nl_buf[];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const RepDev& Rp = reps[ion_rep[i]];
    near_list_one<R>(Rp.g, P, i, n, sxyzq, sxyzf, bin_start + Rp.bin_off, list, count,
                     nl_buf + threadIdx.x, blockDim.x);
}

// The list pass for search radii of 1 to 3 bins (larger radii are rejected up front).
static int launch_near_list(const NearDev& P, int n, int T, hipStream_t s, const GridDev* g,
                            const RepDev* reps, const int* ion_rep, const double4* sxyzq,
                            const float4* sxyzf, const int* bin_start, int* list, int* count) {
    if (P.R < 1 || P.R > 3 || T > 256) return DISCOS_E_ARG;
    const size_t lds = (size_t)NL_SLAB_RUNS(P.R) * T * sizeof(int2);
    const int nb = (n + T - 1) / T;
#define NL_LAUNCH(RR)                                                                           \
    if (g)                                                                                      \
        near_list_kernel<RR><<<nb, T, lds, s>>>(*g, P, n, sxyzq, sxyzf, bin_start, list, count); \
    else                                                                                        \
        near_list_batch_kernel<RR><<<nb, T, lds, s>>>(reps, ion_rep, P, n, sxyzq, sxyzf,        \
                                                      bin_start, list, count);
    if (P.R == 1) {
        NL_LAUNCH(1)
    } else if (P.R == 2) {
        NL_LAUNCH(2)
    } else {
        NL_LAUNCH(3)
    }
#undef NL_LAUNCH
    return DISCOS_OK;
}

// Pair forces of ion i from its list (or, when the list overflowed, from a direct
// walk of the cell list), plus the 9-3 wall force.
__device__ __forceinline__ void list_force(int i, int n, double4 me, int spi,
                                           const double4* __restrict__ sxyzq,
                                           const int* __restrict__ ssp,
                                           const int* __restrict__ bin_start,
                                           const int* __restrict__ list, int cnt, const GridDev& g,
                                           const NearDev& P, double& Fx, double& Fy, double& Fz) {
    const double xi = me.x, yi = me.y, zi = me.z, qi = me.w;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (cnt <= P.cap) {
        const double r2lj = P.rsearch * P.rsearch * (1.0 + 1e-12);
        const int4* chunks = reinterpret_cast<const int4*>(list);
        // the next chunk's entries load while this chunk's pairs are evaluated
        int4 chn = cnt > 0 ? chunks[i] : make_int4(0, 0, 0, 0);
        for (int k4 = 0; k4 < cnt; k4 += 4) {
            const int4 ch = chn;
            if (k4 + 4 < cnt) chn = chunks[(size_t)((k4 >> 2) + 1) * n + i];
            const int m4 = min(4, cnt - k4);
            // the four gathers are issued together (unused slots read the ion itself)
            double4 ob[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = u == 0 ? ch.x : (u == 1 ? ch.y : (u == 2 ? ch.z : ch.w));
                ob[u] = sxyzq[u < m4 ? (e & 0x3FFFFFF) : i];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u >= m4) break;
                const int e = u == 0 ? ch.x : (u == 1 ? ch.y : (u == 2 ? ch.z : ch.w));
                const int j = e & 0x3FFFFFF;
                const int mode = (e >> 30) & 3;
                const double4 o = ob[u];
                const double dx = (xi - shift_of((e >> 26) & 3, g.Lx)) - o.x;
                const double dy = (yi - shift_of((e >> 28) & 3, g.Ly)) - o.y;
                const double dz = mode == 0 ? zi - o.z : (mode == 1 ? zi + o.z : zi - (2.0 * g.Lz - o.z));
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double sg = mode == 0 ? 1.0 : (mode == 1 ? P.s_lo : P.s_hi);
                // the list is a superset (FP32 filter): the exact FP64 tests decide, and a
                // pair at zero separation has no direction and contributes nothing
                if (r2 < P.psi2 && r2 > 0.0) es_pair_r2(dx, dy, dz, r2, qi * (sg * o.w), P, fx, fy, fz);
                if (P.lj_on && mode == 0 && r2 < r2lj && r2 > 0.0) lj_pair(dx, dy, dz, spi, ssp[j], P, fx, fy, fz);
            }
        }
    } else {
        near_force_global(i, me, spi, sxyzq, ssp, bin_start, g, P, fx, fy, fz);
    }
    if (P.wall_on) fz += -du93(zi, P) + du93(g.Lz - zi, P);
    Fx = fx;
    Fy = fy;
    Fz = fz;
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
                                           const double* __restrict__ fp, int64_t fstride,
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
};

__global__ void __launch_bounds__(256)
near_eval_kernel(GridDev g, NearDev P, int n, const double4* __restrict__ sxyzq,
                 const int* __restrict__ ssp, const int* __restrict__ bin_start,
                 const int* __restrict__ list, const int* __restrict__ count,
                 const int* __restrict__ perm, double* __restrict__ out, int64_t stride,
                 int scatter, int* __restrict__ flags, FusedUpdate U) {
    __shared__ double tab[NL_TAB];
    const int nt = min(P.tablen, NL_TAB);
    for (int k = threadIdx.x; k < nt; k += blockDim.x) tab[k] = P.tab[k];
    __syncthreads();
    P.tab = tab;
    const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 me = sxyzq[i];
    if (!pos_ok(g, me.x, me.y, me.z)) {
        if (U.pos)
            update_with_force(g, U.Dd, i, me, ssp[i], U.sid[i], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, U.pos, n,
                              U.q, U.id, U.sp, flags);
        return;
    }
    int spi = 0;
    if (P.lj_on) {
        spi = ssp[i];
        if (spi < 0 || spi >= max(P.nsp, 1)) set_flag(flags, DISCOS_FLAG_BAD_SPECIES);
    }
    double Fx, Fy, Fz;
    list_force(i, n, me, spi, sxyzq, ssp, bin_start, list, count[i], g, P, Fx, Fy, Fz);
    if (U.pos) {
        update_with_force(g, U.Dd, i, me, ssp[i], U.sid[i], out[i] + Fx, out[i + stride] + Fy,
                          out[i + 2 * stride] + Fz, 0.0, 0.0, 0.0, U.pos, n, U.q, U.id, U.sp, flags);
        return;
    }
    const int o = scatter ? perm[i] : i;
    out[o] += Fx;
    out[o + stride] += Fy;
    out[o + 2 * stride] += Fz;
}

__global__ void __launch_bounds__(256)
near_eval_batch_kernel(const RepDev* __restrict__ reps, const int* __restrict__ ion_rep, NearDev P,
                       int n, const double4* __restrict__ sxyzq, const int* __restrict__ ssp,
                       const int* __restrict__ bin_start, const int* __restrict__ list,
                       const int* __restrict__ count, double* __restrict__ out,
                       int* __restrict__ flags) {
    __shared__ double tab[NL_TAB];
    const int nt = min(P.tablen, NL_TAB);
    for (int k = threadIdx.x; k < nt; k += blockDim.x) tab[k] = P.tab[k];
    __syncthreads();
    P.tab = tab;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const RepDev& R = reps[ion_rep[i]];
    const GridDev g = R.g;
    P.s_lo = R.s_lo;
    P.s_hi = R.s_hi;
    const double4 me = sxyzq[i];
    if (!pos_ok(g, me.x, me.y, me.z)) return;
    int spi = 0;
    if (P.lj_on) {
        spi = ssp[i];
        if (spi < 0 || spi >= max(P.nsp, 1)) set_flag(flags, DISCOS_FLAG_BAD_SPECIES);
    }
    double Fx, Fy, Fz;
    list_force(i, n, me, spi, sxyzq, ssp, bin_start + R.bin_off, list, count[i], g, P, Fx, Fy, Fz);
    out[i] += Fx;
    out[i + n] += Fy;
    out[i + 2 * (int64_t)n] += Fz;
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
                      int scatter_to_caller, hipStream_t s, int mark, const DryStepOut* upd) {
    if (n <= 0) return DISCOS_OK;
    const NearDev P = near_of(c, p);
    const int T = 256;
    int rc = launch_near_list(P, n, T, s, &c->gd, nullptr, nullptr, c->sxyzq, c->sxyzf,
                              c->bin_start, c->nlist, c->ncount);
    if (rc) return rc;
    if (mark >= 0) stage_mark(c, mark, s);
    FusedUpdate U{};
    if (upd) {
        U.Dd = dry_of(p, upd->step);
        U.sid = c->sid;
        U.pos = upd->pos;
        U.q = upd->q;
        U.id = upd->id;
        U.sp = upd->sp;
    }
    near_eval_kernel<<<(n + T - 1) / T, T, 0, s>>>(c->gd, P, n, c->sxyzq, c->ssp, c->bin_start,
                                                   c->nlist, c->ncount, c->perm, out, out_stride,
                                                   scatter_to_caller, c->flags, U);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

__global__ void dry_update_kernel(GridDev g, DryDev Dd, int n, const double4* __restrict__ sxyzq,
                                  const int* __restrict__ sid, const int* __restrict__ ssp,
                                  const double* __restrict__ fp, int64_t fstride,
                                  const double* __restrict__ vw,
                                  double* __restrict__ pos, int64_t pstride, double* __restrict__ q,
                                  int* __restrict__ id, int* __restrict__ sp,
                                  int* __restrict__ flags) {
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= n) return;
    update_one(g, Dd, gi, sxyzq, sid, ssp, fp, fstride, vw, pos, pstride, q, id, sp, flags);
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
    update_one(R.g, Dd, gi, sxyzq, sid, ssp, fp, n, nullptr, pos, n, q, id, sp, flags);
}

__global__ void step_advance_kernel(uint64_t* step) { *step += 1; }
__global__ void step_set_kernel(uint64_t* step, uint64_t v) { *step = v; }

int batch_near(Batch* b, hipStream_t s) {
    const int n = (int)b->n_tot;
    if (n == 0) return DISCOS_OK;
    NearDev P = near_of_h(b->h, &b->p);
    P.cap = b->nl_cap;
    const int T = b->cfg.ion_block;
    int rc = launch_near_list(P, n, T, s, nullptr, b->reps_d, b->ion_rep, b->sxyzq, b->sxyzf,
                              b->bin_start, b->nlist, b->ncount);
    if (rc) return rc;
    near_eval_batch_kernel<<<(n + T - 1) / T, T, 0, s>>>(b->reps_d, b->ion_rep, P, n, b->sxyzq,
                                                         b->ssp, b->bin_start, b->nlist, b->ncount,
                                                         b->fp, b->flags);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
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
                  double* pos, double* q, int* id, int* sp, hipStream_t s) {
    if (n <= 0) return DISCOS_OK;
    const DryDev Dd = dry_of(p, step);
    dry_update_kernel<<<(n + 255) / 256, 256, 0, s>>>(c->gd, Dd, n, c->sxyzq, c->sid, c->ssp, c->fp,
                                                      c->n_max, vwet, pos, n, q, id, sp, c->flags);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
