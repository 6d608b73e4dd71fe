// C ABI of the DISCOS core: argument validation, context scratch, and the order of
// the kernels in each call.  Everything here runs on the host and only enqueues work.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.h"

using discos::Ctx;

struct discos_ctx : public Ctx {};

namespace discos {

WallDev wall_of(const discos_params* p) {
    WallDev w;
    w.type[0] = p->bc_type[0];
    w.type[1] = p->bc_type[1];
    w.value[0] = p->bc_value[0];
    w.value[1] = p->bc_value[1];
    w.eps = p->eps;
    w.map[0] = p->bc_type_map[0];
    w.map[1] = p->bc_type_map[1];
    return w;
}

int near_radius_bins(const Ctx* c, const discos_params* p);

}  // namespace discos

namespace {

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

int fail(discos_ctx* c, int code, const char* msg) {
    if (c) c->err = msg;
    return code;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Checks shared by every call that reads discos_params.
int check_es_params(discos_ctx* c, const discos_params* p) {
    if (!p) return fail(c, DISCOS_E_ARG, "params is null");
    if (!finite_pos(p->eps)) return fail(c, DISCOS_E_ARG, "eps must be positive");
    for (int w = 0; w < 2; ++w)
        if (p->bc_type[w] != DISCOS_BC_DIRICHLET && p->bc_type[w] != DISCOS_BC_NEUMANN)
            return fail(c, DISCOS_E_ARG, "bc_type must be DISCOS_BC_DIRICHLET or DISCOS_BC_NEUMANN");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->e_ext[k])) return fail(c, DISCOS_E_ARG, "e_ext must be finite");
    return DISCOS_OK;
}

int check_near_params(discos_ctx* c, const discos_params* p, const int32_t* species) {
    int rc = check_es_params(c, p);
    if (rc) return rc;
    if (!finite_pos(p->psi)) return fail(c, DISCOS_E_ARG, "psi must be positive");
    if (!p->p3m_table || p->p3m_len < 2 || !finite_pos(p->p3m_dr))
        return fail(c, DISCOS_E_ARG, "p3m table missing or malformed");
    if (p->psi / c->grid.h / p->p3m_dr > (double)(p->p3m_len - 1))
        return fail(c, DISCOS_E_ARG, "p3m table does not reach psi");
    if (p->psi / c->grid.h / p->p3m_dr + 2.0 > 320.0)
        return fail(c, DISCOS_E_ARG, "p3m table finer than 320 entries up to psi");
    if (p->wall_on && (!finite_pos(p->wall_sigma) || !std::isfinite(p->wall_xi) ||
                       !finite_pos(p->wall_cut)))
        return fail(c, DISCOS_E_ARG, "wall potential parameters invalid");
    if (p->lj_on) {
        if (!p->lj_sigma || !p->lj_xi || p->nspecies < 1 || !finite_pos(p->lj_cut_factor) ||
            !finite_pos(p->lj_range))
            return fail(c, DISCOS_E_ARG, "LJ parameters invalid");
        if (!species) return fail(c, DISCOS_E_ARG, "LJ needs species");
    }
    const int R = discos::near_radius_bins(c, p);
    if (R > 3) return fail(c, DISCOS_E_ARG, "near-field search radius above 6 h");
    if (2 * R + 1 > c->gd.nbx || 2 * R + 1 > c->gd.nby)
        return fail(c, DISCOS_E_SHAPE,
                    "cutoff too large for the periodic box (need nx/2, ny/2 >= 2 ceil(psi/2h) + 1)");
    return DISCOS_OK;
}

// The wall type maps of p, read on the host (the stream is synchronised first): every
// entry must be a DISCOS_BC_* type.  q receives p with bc_type[w] replaced by the type of
// a uniform map, or for a wall whose columns differ by the preconditioner's reference
// type (Dirichlet); c->wm_mixed records whether a wall's columns differ.
int read_wall_maps(discos_ctx* c, const discos_params* p, hipStream_t s, discos_params& q) {
    q = *p;
    c->wm_mixed = 0;
    c->wm_ref[0] = p->bc_type[0];
    c->wm_ref[1] = p->bc_type[1];
    if (!p->bc_type_map[0] && !p->bc_type_map[1]) return DISCOS_OK;
    const size_t ncol = (size_t)c->gd.nx * c->gd.ny;
    std::vector<int32_t> m(ncol);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(c, DISCOS_E_HIP, "stream failed");
    for (int w = 0; w < 2; ++w) {
        if (!p->bc_type_map[w]) continue;
        if (hipMemcpy(m.data(), p->bc_type_map[w], ncol * sizeof(int32_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return fail(c, DISCOS_E_HIP, "reading a wall type map failed");
        size_t nd = 0, nn = 0;
        for (size_t k = 0; k < ncol; ++k) {
            nd += m[k] == DISCOS_BC_DIRICHLET;
            nn += m[k] == DISCOS_BC_NEUMANN;
        }
        if (nd + nn != ncol) return fail(c, DISCOS_E_ARG, "bc_type_map entries must be DISCOS_BC_*");
        q.bc_type[w] = nd > 0 ? DISCOS_BC_DIRICHLET : DISCOS_BC_NEUMANN;
        c->wm_ref[w] = q.bc_type[w];
        if (nd > 0 && nn > 0) c->wm_mixed = 1;
        // the direct solve of walls of mixed type depends on the maps' contents
        if (c->wm_host[w] != m) {
            c->wm_host[w] = m;
            ++c->wm_gen;
        }
    }
    for (int w = 0; w < 2; ++w)
        if (!p->bc_type_map[w] && !c->wm_host[w].empty()) {
            c->wm_host[w].clear();
            ++c->wm_gen;
        }
    return DISCOS_OK;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n from the
// three-term recurrence, started at the Chebyshev-like guess cos(pi (k - 1/4) / (n + 1/2))).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wt) {
    x.assign(n, 0.0);
    wt.assign(n, 0.0);
    for (int k = 0; k < (n + 1) / 2; ++k) {
        double z = std::cos(M_PI * (k + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[k] = -z;
        x[n - 1 - k] = z;
        wt[k] = wt[n - 1 - k] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Integral of exp(beta (sqrt(1 - (z / alpha)^2) - 1)) over (-alpha, alpha), in cells
// (App. B, eq eskernel): with z = alpha sin(theta) the integrand becomes
// alpha exp(beta (cos(theta) - 1)) cos(theta) on (-pi/2, pi/2), analytic, so composite
// Gauss-Legendre (32 panels of 24 nodes) reaches rounding level for beta <= 100.
double esc_integral(double w, double beta) {
    std::vector<double> gx, gw;
    gauss_legendre(24, gx, gw);
    const double alpha = 0.5 * w;
    const int panels = 32;
    const double hw = M_PI / panels;
    double sum = 0.0;
    for (int pnl = 0; pnl < panels; ++pnl) {
        const double c0 = -0.5 * M_PI + (pnl + 0.5) * hw;
        double ps = 0.0;
        for (size_t k = 0; k < gx.size(); ++k) {
            const double th = c0 + 0.5 * hw * gx[k];
            const double ct = std::cos(th);
            ps += gw[k] * std::exp(beta * (ct - 1.0)) * ct;
        }
        sum += 0.5 * hw * ps;
    }
    return alpha * sum;
}

// Wall types of the hydrodynamic calls (eq fluidbc): checked, then kept as the image
// signs of the tangential velocity in the context's grid descriptor, which every
// hydrodynamic kernel launched by this call receives.
int set_hydro_walls(discos_ctx* c, const discos_params* p) {
    for (int w = 0; w < 2; ++w)
        if (p->hydro_bc[w] != DISCOS_HYDRO_NOSLIP && p->hydro_bc[w] != DISCOS_HYDRO_SLIP)
            return fail(c, DISCOS_E_ARG, "hydro_bc must be DISCOS_HYDRO_NOSLIP or DISCOS_HYDRO_SLIP");
    c->gd.tsg[0] = p->hydro_bc[0] == DISCOS_HYDRO_SLIP ? 1.0 : -1.0;
    c->gd.tsg[1] = p->hydro_bc[1] == DISCOS_HYDRO_SLIP ? 1.0 : -1.0;
    return DISCOS_OK;
}

template <class T>
T* carve(char*& cur, size_t count) {
    T* p = reinterpret_cast<T*>(cur);
    size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    cur += bytes;
    return p;
}

size_t carve_bytes(size_t count, size_t elem) { return (count * elem + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int discos_create(const discos_grid* grid, int64_t n_max, uint32_t flags, discos_ctx** out) {
    (void)flags;
    if (!grid || !out) return DISCOS_E_ARG;
    *out = nullptr;
    if (!pow2_in(grid->nx, 8, 1024) || !pow2_in(grid->ny, 8, 1024) || grid->nz < 4 ||
        grid->nz > 8192 || !finite_pos(grid->h))
        return DISCOS_E_SHAPE;
    if (n_max < 0 || n_max >= ((int64_t)1 << 26)) return DISCOS_E_SHAPE;
    discos_ctx* c = new (std::nothrow) discos_ctx();
    if (!c) return DISCOS_E_HIP;
    c->grid = *grid;
    c->n_max = n_max;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return DISCOS_E_HIP;
    }
    discos::GridDev& g = c->gd;
    g.nx = grid->nx;
    g.ny = grid->ny;
    g.nz = grid->nz;
    g.nxh = grid->nx / 2 + 1;
    g.h = grid->h;
    g.inv_h = 1.0 / grid->h;
    g.Lx = grid->nx * grid->h;
    g.Ly = grid->ny * grid->h;
    g.Lz = grid->nz * grid->h;
    g.lb = DISCOS_LB;
    g.nbx = grid->nx / DISCOS_BIN;
    g.nby = grid->ny / DISCOS_BIN;
    g.nbz = (grid->nz + DISCOS_BIN - 1) / DISCOS_BIN;
    c->ncell = (int64_t)g.nx * g.ny * g.nz;
    c->nface_z = (int64_t)g.nx * g.ny * (g.nz + 1);
    c->nmode = (int64_t)g.nxh * g.ny;
    c->nbins = (int64_t)g.nbx * g.nby * g.nbz;
    const int64_t nm = std::max<int64_t>(n_max, 1);
    const int64_t nblk = (c->nbins + 1023) / 1024 + 1;
    const int64_t nspec = c->nmode * g.nz;
    size_t bytes = 0;
    bytes += carve_bytes(nm, sizeof(double4));         // sxyzq
    bytes += carve_bytes(3 * nm, sizeof(double));      // fp
    bytes += carve_bytes(3 * nm, sizeof(double));      // fnear
    bytes += 5 * carve_bytes(nm, sizeof(int));         // sid ssp perm ion_bin ion_rank
    bytes += carve_bytes(c->nbins, sizeof(int));
    bytes += carve_bytes(c->nbins + 1, sizeof(int));
    bytes += carve_bytes(nblk, sizeof(int));
    bytes += 2 * carve_bytes(c->ncell, sizeof(double)); // rho phi
    bytes += carve_bytes(nspec, sizeof(double2));
    bytes += carve_bytes(nspec, sizeof(double));
    bytes += carve_bytes(g.nx / 2, sizeof(double2));
    bytes += carve_bytes(g.ny / 2, sizeof(double2));
    bytes += carve_bytes(64, sizeof(int));
    bytes += carve_bytes(3 * PART_MAX, sizeof(double));                 // reduction partials
    bytes += carve_bytes(2 * (size_t)g.nx * g.ny, sizeof(double));     // wall adjoints
    const size_t ncap = 6 * (size_t)g.nxh * g.ny + 12 * (size_t)g.nx * g.ny;
    bytes += carve_bytes(2 * (size_t)c->ncell, sizeof(double)) + carve_bytes(ncap, sizeof(double)) +
             carve_bytes(8, sizeof(double));  // walls of mixed type
    // the near field's padded cell list, sized for search radii up to 3 bins
    const int64_t nl_bins = discos::near_list_bins(g, 3);
    const int64_t nl_cap = discos::near_list_entries(g, n_max);
    bytes += carve_bytes(nl_bins, sizeof(int)) + carve_bytes(nl_bins + 1, sizeof(int));
    bytes += carve_bytes(nl_bins / 1024 + 2, sizeof(int));
    bytes += carve_bytes(nl_cap, sizeof(double4)) + carve_bytes(nl_cap, sizeof(float4));
    bytes += carve_bytes(nl_cap, sizeof(int));
    if (hipMalloc(&c->pool, bytes) != hipSuccess) {
        delete c;
        return DISCOS_E_HIP;
    }
    c->pool_bytes = bytes;
    char* cur = static_cast<char*>(c->pool);
    c->sxyzq = carve<double4>(cur, nm);
    c->fp = carve<double>(cur, 3 * nm);
    c->fnear = carve<double>(cur, 3 * nm);
    c->sid = carve<int>(cur, nm);
    c->ssp = carve<int>(cur, nm);
    c->perm = carve<int>(cur, nm);
    c->ion_bin = carve<int>(cur, nm);
    c->ion_rank = carve<int>(cur, nm);
    c->bin_count = carve<int>(cur, c->nbins);
    c->bin_start = carve<int>(cur, c->nbins + 1);
    c->scan_tmp = carve<int>(cur, nblk);
    c->rho = carve<double>(cur, c->ncell);
    c->phi = carve<double>(cur, c->ncell);
    c->spec = carve<double2>(cur, nspec);
    c->cprime = carve<double>(cur, nspec);
    c->tw_x = carve<double2>(cur, g.nx / 2);
    c->tw_y = carve<double2>(cur, g.ny / 2);
    c->flags = carve<int>(cur, 64);
    c->part = carve<double>(cur, 3 * PART_MAX);
    c->bcg = carve<double>(cur, 2 * (size_t)g.nx * g.ny);
    c->pcg = carve<double>(cur, 2 * (size_t)c->ncell);
    c->cap = carve<double>(cur, ncap);
    c->cap_key = -1;
    c->pcg_s = carve<double>(cur, 8);
    c->wm_mixed = 0;
    c->wm_ref[0] = c->wm_ref[1] = DISCOS_BC_DIRICHLET;
    c->nl.count = carve<int>(cur, nl_bins);
    c->nl.start = carve<int>(cur, nl_bins + 1);
    c->nl.tmp = carve<int>(cur, nl_bins / 1024 + 2);
    c->nl.xyzq = carve<double4>(cur, nl_cap);
    c->nl.xyzf = carve<float4>(cur, nl_cap);
    c->nl.sp = carve<int>(cur, nl_cap);
    c->nl.cap = nl_cap;
    c->nl.bins_cap = nl_bins;
    // twiddles exp(-2 pi i k / N)
    std::vector<double2> tw(std::max(g.nx, g.ny) / 2);
    for (int pass = 0; pass < 2; ++pass) {
        const int N = pass == 0 ? g.nx : g.ny;
        for (int k = 0; k < N / 2; ++k) {
            const double a = 2.0 * M_PI * (double)k / (double)N;
            tw[k] = make_double2(std::cos(a), -std::sin(a));
        }
        if (hipMemcpy(pass == 0 ? c->tw_x : c->tw_y, tw.data(), (N / 2) * sizeof(double2),
                      hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(c->pool);
            delete c;
            return DISCOS_E_HIP;
        }
    }
    // flags, and the bin counts (the scan that reads them clears them again)
    if (hipMemset(c->flags, 0, 64 * sizeof(int)) != hipSuccess ||
        hipMemset(c->bin_count, 0, c->nbins * sizeof(int)) != hipSuccess) {
        (void)hipFree(c->pool);
        delete c;
        return DISCOS_E_HIP;
    }
    c->hydro = 0;
    if (flags & DISCOS_CREATE_HYDRO) {
        const size_t ncell = (size_t)c->ncell, nlev = (size_t)c->nface_z;
        const size_t nsp = (size_t)g.nxh * g.ny;
        size_t hb = 0;
        hb += carve_bytes(nsp * (4 * (size_t)g.nz + 1), sizeof(double2));  // u v w p spectra
        hb += carve_bytes(14 * (size_t)g.nz * nsp, sizeof(double));         // mode factors
        hb += carve_bytes(4 * ncell, sizeof(double));                       // stress diag + xy
        hb += carve_bytes(2 * nlev, sizeof(double));                        // stress xz yz
        hb += 2 * carve_bytes(2 * ncell + nlev, sizeof(double));            // hvel, hfor
        hb += carve_bytes(3 * nm, sizeof(double));                          // hvi
        hb += carve_bytes(4 * (DISCOS_HY_MAXSP + 1), sizeof(double));        // kernel table
        void* hp = nullptr;
        if (hipMalloc(&hp, hb) != hipSuccess) {
            (void)hipFree(c->pool);
            delete c;
            return DISCOS_E_HIP;
        }
        c->hpool = hp;
        char* hc = static_cast<char*>(hp);
        c->hspec = carve<double2>(hc, nsp * (4 * (size_t)g.nz + 1));
        c->hfac = carve<double>(hc, 14 * (size_t)g.nz * nsp);
        c->hz_diag = carve<double>(hc, 4 * ncell);
        c->hz_edge = carve<double>(hc, 2 * nlev);
        c->hvel = carve<double>(hc, 2 * ncell + nlev);
        c->hfor = carve<double>(hc, 2 * ncell + nlev);
        c->hvi = carve<double>(hc, 3 * nm);
        c->hy_tab = carve<double>(hc, 4 * (DISCOS_HY_MAXSP + 1));
        c->gd.tsg[0] = c->gd.tsg[1] = -1.0;  // no-slip until a call says otherwise
        // every species on the 4-point Peskin kernel (rows of zeros: w = 0); the Stokes
        // mode factorisation of this grid
        if (hipMemset(c->hy_tab, 0, 4 * (DISCOS_HY_MAXSP + 1) * sizeof(double)) != hipSuccess ||
            discos::stokes_factor(c, nullptr) != DISCOS_OK || hipDeviceSynchronize() != hipSuccess) {
            (void)hipFree(hp);
            (void)hipFree(c->pool);
            delete c;
            return DISCOS_E_HIP;
        }
        c->hydro = 1;
    }
    c->zg_key = -1;
    c->cl_gen = 0;
    c->ef_gen = ~(uint64_t)0;  // no forward list yet
    c->ef_n = -1;
    c->ef_wq = 0.0;
    c->mx_iters = 0;
    c->mx_iterative = (flags & DISCOS_CREATE_MIXED_ITERATIVE) ? 1 : 0;
    c->serial = (flags & DISCOS_CREATE_SERIAL) ? 1 : 0;
    c->cap_nd = -1;
    c->hy_km = 0;
    if (!c->hydro) c->hy_tab = nullptr;
    c->last_stream = nullptr;
    c->err = "";
    c->profile = 0;
    c->prof_stages = 0;
    c->prof_marks = 0;
    c->prof_steps = 0;
    c->ev = nullptr;
    // the dry step's near field runs on a stream of its own beside the grid stages (default
    // priority; fork and join by events, so the step is also capturable into a graph)
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        (void)discos_destroy(c);
        return DISCOS_E_HIP;
    }
    *out = c;
    return DISCOS_OK;
}

int discos_destroy(discos_ctx* c) {
    if (!c) return DISCOS_E_ARG;
    // everything is released even if the device reports an error on the way
    bool ok = hipDeviceSynchronize() == hipSuccess;
    if (c->ev) {
        for (size_t k = 0; k < (size_t)PROF_MAX * (DISCOS_NSTAGE + 1); ++k)
            ok = (hipEventDestroy(c->ev[k]) == hipSuccess) && ok;
        delete[] c->ev;
    }
    if (c->ev_side) {
        for (size_t k = 0; k < PROF_MAX; ++k) ok = (hipEventDestroy(c->ev_side[k]) == hipSuccess) && ok;
        delete[] c->ev_side;
    }
    if (c->ev_fork) ok = (hipEventDestroy(c->ev_fork) == hipSuccess) && ok;
    if (c->ev_join) ok = (hipEventDestroy(c->ev_join) == hipSuccess) && ok;
    if (c->side) ok = (hipStreamDestroy(c->side) == hipSuccess) && ok;
    ok = (hipFree(c->pool) == hipSuccess) && ok;
    if (c->hydro) ok = (hipFree(c->hpool) == hipSuccess) && ok;
    ok = discos::release_dense_capacitance(c) && ok;
    delete c;
    return ok ? DISCOS_OK : DISCOS_E_HIP;
}

int discos_spread(discos_ctx* c, int op, int64_t n, const double* pos, const double* w,
                  const discos_params* p, double* out, void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    const int base = op & 0xFF;
    const int add_bc = (op & DISCOS_SPREAD_ADD_BC) ? 1 : 0;
    if (n < 0 || n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
    if (!out || (n > 0 && (!pos || !w))) return fail(c, DISCOS_E_ARG, "null array");
    int rc = check_es_params(c, p);
    if (rc) return rc;
    if (base == DISCOS_SPREAD_CHARGE) {
        rc = discos::build_cell_list(c, (int)n, pos, pos + n, pos + 2 * n, w, nullptr, nullptr, s);
        if (rc) return fail(c, rc, "cell list launch failed");
        rc = discos::spread_charge_sorted(c, p, add_bc, out, s);
        return rc ? fail(c, rc, "spread launch failed") : DISCOS_OK;
    }
    if (base == DISCOS_SPREAD_FORCE) {
        if (add_bc) return fail(c, DISCOS_E_ARG, "DISCOS_SPREAD_ADD_BC applies to charges only");
        rc = set_hydro_walls(c, p);
        if (rc) return rc;
        rc = discos::build_cell_list(c, (int)n, pos, pos + n, pos + 2 * n, nullptr, nullptr, nullptr,
                                     s, w, n);
        if (rc) return fail(c, rc, "cell list launch failed");
        rc = discos::spread_force_sorted(c, out, s);
        return rc ? fail(c, rc, "spread launch failed") : DISCOS_OK;
    }
    return fail(c, DISCOS_E_ARG, "unknown spread op");
}

int discos_solve_poisson(discos_ctx* c, const double* rhs, const discos_params* p, double* phi,
                         void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (!rhs || !phi) return fail(c, DISCOS_E_ARG, "null array");
    int rc = check_es_params(c, p);
    if (rc) return rc;
    discos_params pm;
    rc = read_wall_maps(c, p, s, pm);
    if (rc) return rc;
    rc = discos::solve_poisson(c, rhs, &pm, phi, s);
    if (rc == DISCOS_E_NOT_CONVERGED) return fail(c, rc, "mixed-wall Poisson solve did not converge");
    return rc ? fail(c, rc, "poisson launch failed") : DISCOS_OK;
}

int discos_solve_stokes(discos_ctx* c, const double* f, const discos_params* p, uint64_t step,
                        int flags, double* v, double* pres, void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (!c->hydro) return fail(c, DISCOS_E_ARG, "context created without DISCOS_CREATE_HYDRO");
    if (!f || !v || !p) return fail(c, DISCOS_E_ARG, "null array");
    if (!finite_pos(p->eta)) return fail(c, DISCOS_E_ARG, "eta must be positive");
    const int noise = (flags & DISCOS_STOKES_NOISE) ? 1 : 0;
    if (noise && (!finite_pos(p->kT) || !finite_pos(p->dt)))
        return fail(c, DISCOS_E_ARG, "noise needs kT > 0 and dt > 0");
    const size_t total = 2 * (size_t)c->ncell + (size_t)c->nface_z;
    if (v < f + total && f < v + total) return fail(c, DISCOS_E_ARG, "f and v overlap");
    int rc = set_hydro_walls(c, p);
    if (rc) return rc;
    rc = discos::solve_stokes(c, f, p, step, noise, v, pres, s);
    return rc ? fail(c, rc, "stokes launch failed") : DISCOS_OK;
}

int discos_interpolate(discos_ctx* c, int op, int64_t n, const double* pos, const double* field,
                       const double* aux, const discos_params* p, double* out, void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (n < 0 || n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
    if (n == 0) return DISCOS_OK;
    if (!pos || !field || !out) return fail(c, DISCOS_E_ARG, "null array");
    int rc = check_es_params(c, p);
    if (rc) return rc;
    if (op == DISCOS_INTERP_E || op == DISCOS_INTERP_FORCE || op == DISCOS_INTERP_PHI) {
        if (op == DISCOS_INTERP_FORCE && !aux) return fail(c, DISCOS_E_ARG, "charges (aux) missing");
        if (n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
        rc = discos::build_cell_list(c, (int)n, pos, pos + n, pos + 2 * n, aux, nullptr, nullptr, s);
        if (!rc) rc = discos::interp_es_sorted(c, op, (int)n, field, p, out, n, 1, s);
        return rc ? fail(c, rc, "interpolation launch failed") : DISCOS_OK;
    }
    if (op == DISCOS_INTERP_VEL) {
        if (n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
        rc = set_hydro_walls(c, p);
        if (rc) return rc;
        rc = discos::build_cell_list(c, (int)n, pos, pos + n, pos + 2 * n, nullptr, nullptr, nullptr, s);
        if (!rc) rc = discos::interp_hy_sorted(c, (int)n, field, out, n, 1, s);
        return rc ? fail(c, rc, "interpolation launch failed") : DISCOS_OK;
    }
    return fail(c, DISCOS_E_ARG, "unknown interpolation op");
}

int discos_set_hydro_kernel(discos_ctx* c, int32_t nspecies, const double* kernel) {
    if (!c) return DISCOS_E_ARG;
    if (!c->hydro) return fail(c, DISCOS_E_ARG, "context created without DISCOS_CREATE_HYDRO");
    if (nspecies < 0 || nspecies > DISCOS_HY_MAXSP)
        return fail(c, DISCOS_E_ARG, "nspecies must lie in [0, DISCOS_HY_MAXSP]");
    if (!kernel) nspecies = 0;
    double tab[4 * (DISCOS_HY_MAXSP + 1)] = {};  // the last row stays Peskin (w = 0)
    int km = 0;
    bool any_esc = false;
    for (int sp = 0; sp < nspecies; ++sp) {
        const double w = kernel[2 * sp], beta = kernel[2 * sp + 1];
        if (w == 0.0) {
            km = std::max(km, 2);
            continue;
        }
        if (!(w >= 2.0 && w <= 8.0 && w == std::floor(w)))
            return fail(c, DISCOS_E_ARG, "kernel width w must be 0 or an integer in [2, 8]");
        if (!(std::isfinite(beta) && beta >= 0.0 && beta <= 100.0))
            return fail(c, DISCOS_E_ARG, "kernel beta must lie in [0, 100]");
        if (c->grid.nz <= (int)w) return fail(c, DISCOS_E_SHAPE, "nz must exceed the kernel width");
        const double norm = esc_integral(w, beta);
        tab[4 * sp + 0] = w;
        tab[4 * sp + 1] = beta;
        tab[4 * sp + 2] = 2.0 / w;
        tab[4 * sp + 3] = 1.0 / norm;
        km = std::max(km, (int)std::ceil(0.5 * w));
        any_esc = true;
    }
    // calls in flight may read the table: let them finish before it changes
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(c->hy_tab, tab, sizeof(tab), hipMemcpyHostToDevice) != hipSuccess)
        return fail(c, DISCOS_E_HIP, "kernel table upload failed");
    c->hy_km = any_esc ? km : 0;
    return DISCOS_OK;
}

int discos_spread_force_species(discos_ctx* c, int64_t n, const double* pos, const double* F,
                                const int32_t* species, const discos_params* p, double* out,
                                void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (!c->hydro) return fail(c, DISCOS_E_ARG, "context created without DISCOS_CREATE_HYDRO");
    if (n < 0 || n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
    if (!out || (n > 0 && (!pos || !F || !species))) return fail(c, DISCOS_E_ARG, "null array");
    int rc = check_es_params(c, p);
    if (!rc) rc = set_hydro_walls(c, p);
    if (rc) return rc;
    rc = discos::build_cell_list(c, (int)n, pos, pos + n, pos + 2 * n, nullptr, nullptr, species, s,
                                 F, n);
    if (rc) return fail(c, rc, "cell list launch failed");
    rc = discos::spread_force_sorted(c, out, s, nullptr, 1);
    return rc ? fail(c, rc, "spread launch failed") : DISCOS_OK;
}

int discos_interpolate_vel_species(discos_ctx* c, int64_t n, const double* pos, const double* v,
                                   const int32_t* species, const discos_params* p, double* out,
                                   void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (!c->hydro) return fail(c, DISCOS_E_ARG, "context created without DISCOS_CREATE_HYDRO");
    if (n < 0 || n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
    if (n == 0) return DISCOS_OK;
    if (!pos || !v || !out || !species) return fail(c, DISCOS_E_ARG, "null array");
    int rc = check_es_params(c, p);
    if (!rc) rc = set_hydro_walls(c, p);
    if (rc) return rc;
    rc = discos::build_cell_list(c, (int)n, pos, pos + n, pos + 2 * n, nullptr, nullptr, species, s);
    if (!rc) rc = discos::interp_hy_sorted(c, (int)n, v, out, n, 1, s, 1);
    return rc ? fail(c, rc, "interpolation launch failed") : DISCOS_OK;
}

int discos_near_field(discos_ctx* c, int64_t n, const double* pos, const double* q,
                      const int32_t* species, const discos_params* p, double* F, void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (n < 0 || n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
    if (n == 0) return DISCOS_OK;
    if (!pos || !q || !F) return fail(c, DISCOS_E_ARG, "null array");
    int rc = check_near_params(c, p, species);
    if (rc) return rc;
    rc = discos::build_cell_list(c, (int)n, pos, pos + n, pos + 2 * n, q, nullptr, species, s);
    if (rc) return fail(c, rc, "cell list launch failed");
    rc = discos::near_field_sorted(c, (int)n, p, F, n, 1, s);
    return rc ? fail(c, rc, "near-field launch failed") : DISCOS_OK;
}

int discos_step(discos_ctx* c, discos_ions* ions, const discos_params* p, uint64_t step, int mode,
                void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (!ions) return fail(c, DISCOS_E_ARG, "ions is null");
    const int64_t n = ions->n;
    if (n < 0 || n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
    if (n > 0 && (!ions->pos || !ions->q || !ions->id || !ions->species))
        return fail(c, DISCOS_E_ARG, "null ion array");
    const int base = mode & 0xF;
    const int rfd = (mode & DISCOS_STEP_RFD) ? 1 : 0;
    if ((mode & ~(0xF | DISCOS_STEP_RFD)) || (base != DISCOS_STEP_DRY && base != DISCOS_STEP_WET))
        return fail(c, DISCOS_E_ARG, "unknown step mode");
    const int wet = base == DISCOS_STEP_WET;
    if (rfd && !wet) return fail(c, DISCOS_E_ARG, "DISCOS_STEP_RFD needs DISCOS_STEP_WET");
    if (wet && !c->hydro) return fail(c, DISCOS_E_ARG, "context created without DISCOS_CREATE_HYDRO");
    int rc = check_near_params(c, p, ions->species);
    if (rc) return rc;
    if (!finite_pos(p->kT) || !finite_pos(p->eta) || !finite_pos(p->dt) || p->nspecies < 1 ||
        !p->radius || !p->mob_coef)
        return fail(c, DISCOS_E_ARG, "dynamics parameters invalid");
    // |delta W / 2| <= 0.05 h * 8.6 (the largest Box-Muller normal of 53-bit uniforms)
    // stays below half a cell, the reach the S^hy tiles assume
    if (rfd && !(finite_pos(p->rfd_delta) && p->rfd_delta <= 0.1 * c->grid.h))
        return fail(c, DISCOS_E_ARG, "rfd_delta must lie in (0, 0.1 h]");
    if (wet) {
        rc = set_hydro_walls(c, p);
        if (rc) return rc;
    }
    discos_params pm;
    rc = read_wall_maps(c, p, s, pm);
    if (rc) return rc;
    p = &pm;
    const int ni = (int)n;
    double* pos = ions->pos;
    discos::stage_mark(c, 0, s);
    rc = discos::build_cell_list(c, ni, pos, pos + n, pos + 2 * n, ions->q, ions->id,
                                 ions->species, s);
    discos::stage_mark(c, 1, s);
    // a dry step: the near field (which needs only the cell list) runs on the side stream
    // while this stream spreads, solves and interpolates; the update then adds the two
    // forces.  Stage marks: the padded list opens on the side stream, which also closes it
    // and the pass (and the two hydrodynamic stages after it, empty); this stream closes
    // the interpolation, then the join (stage 12: the time the grid stages ran past the
    // pass) and the update (stage 13).
    const bool beside = !wet && !c->serial && ni > 0 && !rc;
    if (beside) {
        if (hipEventRecord(c->ev_fork, s) != hipSuccess ||
            hipStreamWaitEvent(c->side, c->ev_fork, 0) != hipSuccess)
            rc = DISCOS_E_HIP;
        discos::stage_open_side(c, 8, c->side);
        if (!rc) rc = discos::near_field_sorted(c, ni, p, c->fnear, c->n_max, 0, c->side, 9,
                                                nullptr, true);
        discos::stage_mark(c, 11, c->side);
        discos::stage_mark(c, 12, c->side);
        if (!rc && hipEventRecord(c->ev_join, c->side) != hipSuccess) rc = DISCOS_E_HIP;
    }
    if (!rc) rc = discos::spread_charge_sorted(c, p, 1, c->rho, s);
    discos::stage_mark(c, 2, s);
    if (!rc) rc = discos::solve_poisson(c, c->rho, p, c->phi, s, 3);
    if (!rc) rc = discos::interp_es_sorted(c, DISCOS_INTERP_FORCE, ni, c->phi, p, c->fp, c->n_max, 0, s);
    discos::stage_mark(c, 8, s);
    // complete the forces in place: fp (grid + applied field) += near field + wall (+ LJ);
    // in a dry step the same pass applies the update from the complete forces
    discos::DryStepOut dry_out{step, pos, ions->q, ions->id, ions->species};
    if (beside) {
        if (!rc && hipStreamWaitEvent(s, c->ev_join, 0) != hipSuccess) rc = DISCOS_E_HIP;
        discos::stage_mark(c, 13, s);
        if (!rc) rc = discos::update_sorted(c, ni, p, step, nullptr, pos, ions->q, ions->id,
                                            ions->species, s, c->fnear);
    } else if (!rc && ni > 0) rc = discos::near_field_sorted(c, ni, p, c->fp, c->n_max, 0, s, 9,
                                                      wet ? nullptr : &dry_out);
    else {
        discos::stage_mark(c, 9, s);
        discos::stage_mark(c, 10, s);
    }
    const double* vwet = nullptr;
    if (wet && !rc && ni > 0) {
        discos::RfdDev rd{};
        if (rfd) {
            rd.sid = c->sid;
            rd.scale = p->kT / p->rfd_delta;
            rd.half = 0.5 * p->rfd_delta;
            rd.seed = p->seed;
            rd.step = step;
        }
        rc = discos::spread_force_sorted(c, c->hfor, s, rfd ? &rd : nullptr, 1, ni);
        discos::stage_mark(c, 11, s);
        if (!rc) rc = discos::solve_stokes(c, c->hfor, p, step, 1, c->hvel, nullptr, s);
        discos::stage_mark(c, 12, s);
        if (!rc) rc = discos::midpoint_velocity(c, ni, c->hvel, p->dt, s, 1);
        discos::stage_mark(c, 13, s);
        vwet = c->hvi;
    } else if (!beside) {
        discos::stage_mark(c, 11, s);
        discos::stage_mark(c, 12, s);
        discos::stage_mark(c, 13, s);
    }
    if (!rc && wet) rc = discos::update_sorted(c, ni, p, step, vwet, pos, ions->q, ions->id, ions->species, s);
    discos::stage_mark(c, 14, s);
    if (c->profile && c->prof_steps < PROF_MAX) ++c->prof_steps;
    return rc ? fail(c, rc, "step launch failed") : DISCOS_OK;
}

int discos_energy_flux(discos_ctx* c, int64_t n, const double* pos, const double* q,
                       const discos_params* p, double* phi, double* out, void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (n < 0 || n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
    if (!phi || !out || (n > 0 && (!pos || !q))) return fail(c, DISCOS_E_ARG, "null array");
    if (p && (p->bc_type_map[0] || p->bc_type_map[1]))
        return fail(c, DISCOS_E_ARG, "the energy / flux adjoint takes uniform walls");
    int rc = check_es_params(c, p);
    if (rc) return rc;
    if (!finite_pos(p->eta)) return fail(c, DISCOS_E_ARG, "eta must be positive (flux weight)");
    const int ni = (int)n;
    c->ef_wq = 0.0;  // set again by a complete forward pass
    rc = discos::build_cell_list(c, ni, pos, pos + n, pos + 2 * n, q, nullptr, nullptr, s);
    c->ef_gen = c->cl_gen;
    c->ef_n = ni;
    if (!rc) rc = discos::spread_charge_sorted(c, p, 1, c->rho, s);
    if (!rc) rc = discos::solve_poisson(c, c->rho, p, phi, s);
    if (!rc && ni > 0)
        rc = discos::interp_es_sorted(c, DISCOS_INTERP_FORCE, ni, phi, p, c->fp, c->n_max, 0, s);
    if (!rc) rc = discos::energy_flux(c, ni, p, phi, out, s);
    return rc ? fail(c, rc, "energy/flux launch failed") : DISCOS_OK;
}

int discos_energy_flux_backward(discos_ctx* c, int64_t n, const double* pos, const double* q,
                                const discos_params* p, const double* phi, const double* g,
                                double* dpos, double* dq, double* dbc_lo, double* dbc_hi,
                                double* de, uint32_t flags, void* stream) {
    if (!c) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (n < 0 || n > c->n_max) return fail(c, DISCOS_E_CAPACITY, "n exceeds n_max");
    if (!phi || !g || (n > 0 && (!pos || !q))) return fail(c, DISCOS_E_ARG, "null array");
    if (p && (p->bc_type_map[0] || p->bc_type_map[1]))
        return fail(c, DISCOS_E_ARG, "the energy / flux adjoint takes uniform walls");
    int rc = check_es_params(c, p);
    if (rc) return rc;
    if (!finite_pos(p->eta)) return fail(c, DISCOS_E_ARG, "eta must be positive (flux weight)");
    const int ni = (int)n;
    // the forward pass's cell list when the caller vouches for unchanged ions and no call
    // has rebuilt it since
    const bool reuse = (flags & DISCOS_ADJ_REUSE_CELLS) && c->ef_gen == c->cl_gen && c->ef_n == ni;
    if (!reuse) rc = discos::build_cell_list(c, ni, pos, pos + n, pos + 2 * n, q, nullptr, nullptr, s);
    if (!rc) rc = discos::energy_flux_backward(c, ni, p, phi, g, dpos, dq, dbc_lo, dbc_hi, de, reuse, s);
    return rc ? fail(c, rc, "energy/flux backward launch failed") : DISCOS_OK;
}

int discos_profile(discos_ctx* c, int enable) {
    return discos_profile_stages(c, enable ? (1u << DISCOS_NSTAGE) - 1u : 0u);
}

int discos_profile_stages(discos_ctx* c, uint32_t stages) {
    if (!c) return DISCOS_E_ARG;
    stages &= (1u << DISCOS_NSTAGE) - 1u;
    const int enable = stages != 0;
    if (enable && !c->ev) {
        const size_t ne = (size_t)PROF_MAX * (DISCOS_NSTAGE + 1);
        c->ev = new (std::nothrow) hipEvent_t[ne];
        if (!c->ev) return fail(c, DISCOS_E_HIP, "event table");
        for (size_t k = 0; k < ne; ++k)
            if (hipEventCreate(&c->ev[k]) != hipSuccess) return fail(c, DISCOS_E_HIP, "event create");
        c->ev_side = new (std::nothrow) hipEvent_t[PROF_MAX];
        if (!c->ev_side) return fail(c, DISCOS_E_HIP, "event table");
        for (size_t k = 0; k < PROF_MAX; ++k)
            if (hipEventCreate(&c->ev_side[k]) != hipSuccess) return fail(c, DISCOS_E_HIP, "event create");
    }
    c->prof_side.assign(PROF_MAX, 0);
    c->profile = enable ? 1 : 0;
    c->prof_stages = stages;
    c->prof_marks = stages | (stages << 1);
    c->prof_steps = 0;
    return DISCOS_OK;
}

int discos_profile_read(discos_ctx* c, double* ms, int* count) {
    if (!c || !ms || !count) return DISCOS_E_ARG;
    *count = 0;
    if (!c->ev) return fail(c, DISCOS_E_ARG, "profiling was never enabled");
    const int ns = c->prof_steps;
    for (int k = 0; k < DISCOS_NSTAGE; ++k) ms[k] = 0.0;
    if (ns == 0) return DISCOS_OK;
    const int row = DISCOS_NSTAGE + 1;
    // the last step's highest recorded event
    const int kmax = 31 - __builtin_clz(c->prof_marks);
    if (hipEventSynchronize(c->ev[(size_t)(ns - 1) * row + kmax]) != hipSuccess)
        return fail(c, DISCOS_E_HIP, "event sync");
    for (int st = 0; st < ns; ++st)
        for (int k = 0; k < DISCOS_NSTAGE; ++k) {
            if (!((c->prof_stages >> k) & 1u)) continue;
            float t = 0.0f;
            // a stage that ran on the side stream opened there
            const hipEvent_t open = (k == 8 && c->prof_side[st]) ? c->ev_side[st]
                                                                  : c->ev[(size_t)st * row + k];
            if (hipEventElapsedTime(&t, open, c->ev[(size_t)st * row + k + 1]) != hipSuccess)
                return fail(c, DISCOS_E_HIP, "event elapsed");
            ms[k] += t / ns;
        }
    *count = DISCOS_NSTAGE;
    return DISCOS_OK;
}

int discos_check(discos_ctx* c) {
    if (!c) return DISCOS_E_ARG;
    if (hipStreamSynchronize(c->last_stream) != hipSuccess) return fail(c, DISCOS_E_HIP, "sync failed");
    int f = 0;
    if (hipMemcpy(&f, c->flags, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, DISCOS_E_HIP, "flag read failed");
    if (f && hipMemset(c->flags, 0, sizeof(int)) != hipSuccess)
        return fail(c, DISCOS_E_HIP, "flag reset failed");
    if (f & DISCOS_FLAG_NONFINITE) return fail(c, DISCOS_E_NONFINITE, "non-finite position");
    if (f & DISCOS_FLAG_BAD_SPECIES) return fail(c, DISCOS_E_ARG, "species index out of range");
    if (f & DISCOS_FLAG_CAPACITY) return fail(c, DISCOS_E_CAPACITY, "tile candidate rows exceeded");
    if (f & DISCOS_FLAG_NOT_NEUTRAL) return fail(c, DISCOS_E_NOT_NEUTRAL, "system not neutral");
    if (f & DISCOS_FLAG_OUT_OF_DOMAIN) return fail(c, DISCOS_E_OUT_OF_DOMAIN, "ion outside channel");
    return DISCOS_OK;
}

const char* discos_last_error(discos_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

}  // extern "C"
