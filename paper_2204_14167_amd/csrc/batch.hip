// Batches of independent channels: layout, launch order, the captured hipGraph of one
// batched step and the launch-parameter autotuner.  Each channel is exactly the dry
// step of a single context (Sec. II.D stages 1-2, eq ions3); nothing couples channels.
//
// Layout: ions and bins follow the channels' order (channel r owns ion slots
// [off_r, off_r + n_r) and a contiguous range of bins, so one batch-wide counting sort
// keeps every channel's ions inside its own slots); cells, spectra and Thomas scratch
// are grouped by (nx, ny) class so that each class's FFT rows and levels are single
// ranges for one launch.
#include <array>
#include <cmath>
#include <map>
#include <new>

#include "kernels.h"

using discos::Batch;

struct discos_batch : public Batch {};

namespace {

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int fail(discos_batch* b, int code, const char* msg) {
    if (b) b->err = msg;
    return code;
}

size_t carve_bytes(size_t n, size_t elem) { return (n * elem + 255) & ~(size_t)255; }

template <class T>
T* carve(char*& cur, size_t n) {
    T* p = reinterpret_cast<T*>(cur);
    cur += carve_bytes(n, sizeof(T));
    return p;
}

// Tile counts of one channel for a tile of (tx, ty, tz) (tx, ty clipped to the grid).
int tiles_of(const discos_replica& r, int tx, int ty, int tz) {
    return (r.nx / std::min(tx, r.nx)) * (r.ny / std::min(ty, r.ny)) * ((r.nz + tz - 1) / tz);
}

// Releases everything; false if the runtime reported an error on the way.
bool destroy(discos_batch* b) {
    if (!b) return true;
    bool ok = true;
    if (b->exec) ok = (hipGraphExecDestroy(b->exec) == hipSuccess) && ok;
    if (b->graph) ok = (hipGraphDestroy(b->graph) == hipSuccess) && ok;
    if (b->own) ok = (hipStreamDestroy(b->own) == hipSuccess) && ok;
    if (b->pool) ok = (hipFree(b->pool) == hipSuccess) && ok;
    delete b;
    return ok;
}

int run_step(discos_batch* b, double* pos, double* q, int* id, int* sp, hipStream_t s) {
    int rc = discos::batch_cell_list(b, pos, q, id, sp, s);
    if (!rc) rc = discos::batch_spread(b, s);
    if (!rc) rc = discos::batch_poisson(b, s);
    if (!rc) rc = discos::batch_interp(b, s);
    if (!rc) rc = discos::batch_near(b, s);
    if (!rc) rc = discos::batch_update(b, pos, q, id, sp, s);
    return rc;
}

}  // namespace

extern "C" {

// Flag the channels with fewer than thresh ions per 2048 cells for the one-thread-per-ion
// interpolation (stage 0) or spread (stage 1); synchronous copy: at creation and while
// tuning.
static bool set_direct(discos_batch* b, int stage, int thresh) {
    std::vector<int> f(b->ions_per_tile.size(), 0);
    int nf = 0;
    for (size_t r = 0; r < f.size(); ++r)
        if (b->ions_per_tile[r] < thresh) {
            f[r] = 1;
            ++nf;
        }
    (stage == 0 ? b->n_direct : b->n_sdirect) = nf;
    (stage == 0 ? b->cfg.interp_direct : b->cfg.spread_direct) = thresh;
    return hipMemcpy(stage == 0 ? b->idirect : b->sdirect, f.data(), f.size() * sizeof(int),
                     hipMemcpyHostToDevice) == hipSuccess;
}

}  // extern "C"

namespace {

// Grid of channel c with the cell-list bin edge 2^lb cells (the bin fields only).
discos::GridDev bin_grid(const discos_replica& c, double h, int lb) {
    discos::GridDev g{};
    g.nx = c.nx;
    g.ny = c.ny;
    g.nz = c.nz;
    g.h = h;
    g.lb = lb;
    g.nbx = c.nx >> lb;
    g.nby = c.ny >> lb;
    g.nbz = (c.nz + (1 << lb) - 1) >> lb;
    return g;
}

// Bins and padded bins of every channel for the bin edge 2^lb (host side only).
discos::BinLayout bin_layout(const std::vector<discos_replica>& reps, double h,
                             const discos_params* p, int lb) {
    discos::BinLayout L;
    const int count = (int)reps.size();
    L.R = discos::near_radius_bins_h(h, p, lb);
    L.ok = L.R >= 1 && L.R <= 3;
    L.bin_off.assign(count + 1, 0);
    L.pbin_off.assign(count + 1, 0);
    int pmax = 1;
    for (int r = 0; r < count; ++r) {
        const discos_replica& c = reps[r];
        const discos::GridDev g = bin_grid(c, h, lb);
        // the search window of 2R + 1 bins may not wrap onto itself in x or y
        if (2 * L.R + 1 > g.nbx || 2 * L.R + 1 > g.nby) L.ok = false;
        L.bin_off[r + 1] = L.bin_off[r] + g.nbx * g.nby * g.nbz;
        const int64_t pb = discos::near_list_bins(g, std::max(L.R, 1));
        L.pbin_off[r + 1] = L.pbin_off[r] + (int)pb;
        pmax = std::max(pmax, (int)pb);
        L.nl_entries += discos::near_list_entries(g, c.n);
    }
    L.nbins = L.bin_off[count];
    L.pbins = L.pbin_off[count];
    L.pbin_xblocks = std::min((pmax + 255) / 256, 64);
    return L;
}

// Switches the batch to the bin edge 2^lb (a layout whose bins fit the allocation):
// channel grids and first bins on the device, bin counts cleared, a captured graph
// dropped (its launch shapes change).  Synchronous.
bool apply_layout(discos_batch* b, int lb) {
    const discos::BinLayout& L = b->lay[lb];
    const int count = (int)b->reps.size();
    for (int r = 0; r < count; ++r) {
        discos::RepDev& d = b->reps_h[r];
        const discos::GridDev g = bin_grid(b->reps[r], b->h, lb);
        d.g.lb = lb;
        d.g.nbx = g.nbx;
        d.g.nby = g.nby;
        d.g.nbz = g.nbz;
        d.bin_off = L.bin_off[r];
    }
    b->cfg.lb = lb;
    b->nbins_tot = L.nbins;
    b->pbins_tot = L.pbins;
    b->pbin_xblocks = L.pbin_xblocks;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    bool ok = hipDeviceSynchronize() == hipSuccess;
    ok = ok && hipMemcpy(b->reps_d, b->reps_h.data(), count * sizeof(discos::RepDev),
                         hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->pbin_off, L.pbin_off.data(), (count + 1) * sizeof(int),
                         hipMemcpyHostToDevice) == hipSuccess;
    // bin counts start at zero; the scan that reads them clears them again
    ok = ok && hipMemset(b->bin_count, 0, b->lay[1].nbins * sizeof(int)) == hipSuccess;
    return ok;
}

}  // namespace

extern "C" {

int discos_batch_create(const discos_replica* reps, int32_t count, double h, const discos_params* p,
                        discos_batch** out) {
    if (!out) return DISCOS_E_ARG;
    *out = nullptr;
    if (!reps || count < 1 || !p) return DISCOS_E_ARG;
    if (!finite_pos(h) || !finite_pos(p->eps) || !finite_pos(p->psi) || !finite_pos(p->kT) ||
        !finite_pos(p->eta) || !finite_pos(p->dt) || p->nspecies < 1 || !p->radius ||
        !p->p3m_table || p->p3m_len < 2 || !finite_pos(p->p3m_dr))
        return DISCOS_E_ARG;
    for (int w = 0; w < 2; ++w)
        if (p->bc_type[w] != DISCOS_BC_DIRICHLET && p->bc_type[w] != DISCOS_BC_NEUMANN)
            return DISCOS_E_ARG;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->e_ext[k])) return DISCOS_E_ARG;
    if (p->psi / h / p->p3m_dr > (double)(p->p3m_len - 1)) return DISCOS_E_ARG;
    // the entries the cutoff can reach are copied to LDS by the force pass (320 at most)
    if (p->psi / h / p->p3m_dr + 2.0 > 320.0) return DISCOS_E_ARG;
    if (p->lj_on && (!p->lj_sigma || !p->lj_xi || !finite_pos(p->lj_range))) return DISCOS_E_ARG;
    if (p->bc_type_map[0] || p->bc_type_map[1]) return DISCOS_E_ARG;  // channels have uniform walls
    const int Rb = discos::near_radius_bins_h(h, p, DISCOS_LB);
    if (Rb > 3) return DISCOS_E_ARG;
    int64_t n_tot = 0;
    for (int r = 0; r < count; ++r) {
        const discos_replica& c = reps[r];
        if (!pow2_in(c.nx, 8, 1024) || !pow2_in(c.ny, 8, 1024) || c.nz < 4 || c.nz > 4096 || c.n < 0)
            return DISCOS_E_SHAPE;
        if (2 * Rb + 1 > c.nx / DISCOS_BIN || 2 * Rb + 1 > c.ny / DISCOS_BIN) return DISCOS_E_SHAPE;
        if (!c.mob_coef && !p->mob_coef) return DISCOS_E_ARG;
        if (!std::isfinite(c.bc_value[0]) || !std::isfinite(c.bc_value[1])) return DISCOS_E_ARG;
        n_tot += c.n;
    }
    if (n_tot >= (int64_t(1) << 26)) return DISCOS_E_CAPACITY;

    discos_batch* b = new (std::nothrow) discos_batch();
    if (!b) return DISCOS_E_HIP;
    b->R = count;
    b->h = h;
    b->p = *p;
    b->reps.assign(reps, reps + count);
    b->n_tot = n_tot;
    b->cfg = {16, 0, 16, 0, 256, 1 << 30, 24, DISCOS_LB};
    b->next_step = ~uint64_t(0);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        destroy(b);
        return DISCOS_E_HIP;
    }
    // the compute-unit count only sizes the tuning candidates: 256 if it cannot be read
    if (hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        b->ncu <= 0)
        b->ncu = 256;

    // ions and bins in channel order; the bins and the near field's padded bins and copies
    // for both bin edges (2 cells: DISCOS_BIN, the default; 4 cells where every channel is
    // wide enough), buffers sized for the larger of the two
    b->ion_off.assign(count + 1, 0);
    for (int r = 0; r < count; ++r) b->ion_off[r + 1] = b->ion_off[r] + reps[r].n;
    for (int lb = 1; lb <= 2; ++lb) b->lay[lb] = bin_layout(b->reps, h, p, lb);
    const std::vector<int>& bin_off = b->lay[DISCOS_LB].bin_off;
    const std::vector<int>& pbin_off = b->lay[DISCOS_LB].pbin_off;
    b->nbins_tot = b->lay[DISCOS_LB].nbins;
    b->pbins_tot = b->lay[DISCOS_LB].pbins;
    const int64_t nbins_cap = std::max(b->lay[1].nbins, b->lay[2].nbins);
    const int64_t pbins_cap = std::max(b->lay[1].pbins, b->lay[2].ok ? b->lay[2].pbins : 0);
    const int64_t nl_cap = std::max(b->lay[1].nl_entries, b->lay[2].ok ? b->lay[2].nl_entries : 0);
    // cells and spectra by (nx, ny) class
    std::map<std::pair<int, int>, std::vector<int>> cls;
    for (int r = 0; r < count; ++r) cls[{reps[r].nx, reps[r].ny}].push_back(r);
    b->reps_h.resize(count);
    std::vector<int> mode_off(count + 1, 0), mode_rep(count, 0);
    int64_t cell = 0, spec = 0, wall = 0;
    int slot = 0;
    for (auto& kv : cls) {
        discos::BatchClass k{};
        k.nx = kv.first.first;
        k.ny = kv.first.second;
        k.rep_first = slot;
        k.rep_count = (int)kv.second.size();
        k.cell_off = cell;
        k.spec_off = spec;
        for (int r : kv.second) {
            const discos_replica& c = reps[r];
            discos::RepDev& d = b->reps_h[r];
            discos::GridDev& g = d.g;
            g.nx = c.nx;
            g.ny = c.ny;
            g.nz = c.nz;
            g.nxh = c.nx / 2 + 1;
            g.h = h;
            g.inv_h = 1.0 / h;
            g.Lx = c.nx * h;
            g.Ly = c.ny * h;
            g.Lz = c.nz * h;
            g.lb = DISCOS_LB;
            g.nbx = c.nx >> DISCOS_LB;
            g.nby = c.ny >> DISCOS_LB;
            g.nbz = (c.nz + DISCOS_BIN - 1) >> DISCOS_LB;
            d.cell_off = cell;
            d.spec_off = spec;
            d.bin_off = bin_off[r];
            d.ion_off = (int)b->ion_off[r];
            d.n = (int)c.n;
            d.s_lo = p->bc_type[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
            d.s_hi = p->bc_type[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
            d.scale = (h * h / p->eps) / ((double)c.nx * c.ny);
            d.singular = p->bc_type[0] == DISCOS_BC_NEUMANN && p->bc_type[1] == DISCOS_BC_NEUMANN;
            d.nmode = g.nxh * c.ny;
            d.seed = c.seed;
            d.coef = c.mob_coef ? c.mob_coef : p->mob_coef;
            d.w.type[0] = p->bc_type[0];
            d.w.type[1] = p->bc_type[1];
            d.w.eps = p->eps;
            d.w.value[0] = reinterpret_cast<const double*>(wall);  // offsets; rebased below
            d.w.value[1] = reinterpret_cast<const double*>(wall + (int64_t)c.nx * c.ny);
            wall += 2 * (int64_t)c.nx * c.ny;
            cell += (int64_t)c.nx * c.ny * c.nz;
            spec += (int64_t)g.nxh * c.ny * c.nz;
            k.rows += c.ny * c.nz;
            k.levels += c.nz;
            mode_rep[slot] = r;
            mode_off[slot + 1] = mode_off[slot] + d.nmode;
            ++slot;
        }
        b->classes.push_back(k);
    }
    b->ncell_tot = cell;
    b->nspec_tot = spec;
    b->nmode_tot = mode_off[count];
    // z-solve: pivots once per grid shape (channels with nz <= 128), tasks of 16 modes per
    // wavefront grouped by segment length; channels with nz > 128 keep the per-mode
    // Thomas sweep with spectrum-sized scratch
    std::map<std::array<int, 3>, int64_t> zshape;
    int64_t zg_len = 0;
    std::vector<int2> zt[3];
    for (int r = 0; r < count; ++r) {
        const discos_replica& c = reps[r];
        discos::RepDev& d = b->reps_h[r];
        d.zg_off = 0;
        if (d.singular) b->z_singular = true;
        if (c.nz > 128) {
            b->z_legacy = true;
            continue;
        }
        const std::array<int, 3> key{c.nx, c.ny, c.nz};
        auto it = zshape.find(key);
        if (it == zshape.end()) {
            it = zshape.emplace(key, zg_len).first;
            b->zshapes.push_back({(int64_t)c.nx, (int64_t)c.ny, (int64_t)c.nz, zg_len});
            zg_len += (int64_t)c.nz * d.nmode;
        }
        d.zg_off = it->second;
        const int L = (c.nz + 3) / 4;
        const int v = L <= 8 ? 0 : (L <= 16 ? 1 : 2);
        for (int t0 = 0; t0 < d.nmode; t0 += 16) zt[v].push_back(make_int2(r, t0));
    }
    // tile tasks, largest channels first
    std::vector<int> order(count);
    for (int r = 0; r < count; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return (int64_t)reps[a].nx * reps[a].ny * reps[a].nz > (int64_t)reps[c].nx * reps[c].ny * reps[c].nz;
    });
    std::vector<int2> tk[2][2];
    const int tsz[2][2][3] = {{{8, 8, 8}, {16, 16, 16}}, {{8, 8, 8}, {16, 16, 8}}};
    for (int kind = 0; kind < 2; ++kind)
        for (int v = 0; v < 2; ++v)
            for (int r : order) {
                const int nt = tiles_of(reps[r], tsz[kind][v][0], tsz[kind][v][1], tsz[kind][v][2]);
                for (int t = 0; t < nt; ++t) tk[kind][v].push_back(make_int2(r, t));
            }
    // twiddles per distinct axis length
    std::map<int, int> tw_index;
    std::vector<double2> tw_all;
    auto tw_of = [&](int N) {
        auto it = tw_index.find(N);
        if (it != tw_index.end()) return it->second;
        const int at = (int)tw_all.size();
        for (int q = 0; q < N / 2; ++q) {
            const double a = 2.0 * M_PI * (double)q / (double)N;
            tw_all.push_back(make_double2(std::cos(a), -std::sin(a)));
        }
        tw_index[N] = at;
        return at;
    };
    std::vector<std::pair<int, int>> tw_at;
    for (auto& k : b->classes) tw_at.push_back({tw_of(k.nx), tw_of(k.ny)});

    // one allocation
    const size_t n = (size_t)std::max<int64_t>(n_tot, 1);
    const size_t nblk = (size_t)(nbins_cap + 1023) / 1024 + 1;
    size_t bytes = 0;
    bytes += carve_bytes(n, sizeof(double4));
    bytes += carve_bytes(pbins_cap, sizeof(int)) + carve_bytes(pbins_cap + 1, sizeof(int));
    bytes += carve_bytes(pbins_cap / 1024 + 2, sizeof(int)) + carve_bytes(count + 1, sizeof(int));
    bytes += carve_bytes(nl_cap, sizeof(double4)) + carve_bytes(nl_cap, sizeof(float4));
    bytes += carve_bytes(nl_cap, sizeof(int));
    bytes += 6 * carve_bytes(n, sizeof(int));  // sid ssp perm ion_bin ion_rank ion_rep
    bytes += carve_bytes(nbins_cap, sizeof(int)) + carve_bytes(nbins_cap + 1, sizeof(int));
    bytes += carve_bytes(nblk, sizeof(int));
    bytes += 2 * carve_bytes(b->ncell_tot, sizeof(double));
    const int64_t ncp = b->z_legacy ? b->nspec_tot : 1;
    bytes += carve_bytes(b->nspec_tot, sizeof(double2)) + carve_bytes(ncp, sizeof(double));
    bytes += carve_bytes(std::max<int64_t>(zg_len, 1), sizeof(double));
    for (int v = 0; v < 3; ++v) bytes += carve_bytes(std::max<size_t>(zt[v].size(), 1), sizeof(int2));
    bytes += carve_bytes(3 * n, sizeof(double));
    bytes += carve_bytes(64, sizeof(int)) + carve_bytes(1, sizeof(uint64_t));
    bytes += carve_bytes(count + 1, sizeof(int)) + carve_bytes(count, sizeof(int));
    bytes += carve_bytes(count, sizeof(discos::RepDev));
    for (int kind = 0; kind < 2; ++kind)
        for (int v = 0; v < 2; ++v) bytes += carve_bytes(std::max<size_t>(tk[kind][v].size(), 1), sizeof(int2));
    bytes += carve_bytes(std::max<int64_t>(wall, 1), sizeof(double));
    bytes += carve_bytes(tw_all.size(), sizeof(double2));
    bytes += carve_bytes(b->classes.size(), sizeof(discos::FftClassDev));
    bytes += 2 * carve_bytes(count, sizeof(int));  // idirect, sdirect
    if (hipMalloc(&b->pool, bytes) != hipSuccess) {
        destroy(b);
        return DISCOS_E_HIP;
    }
    char* cur = static_cast<char*>(b->pool);
    b->sxyzq = carve<double4>(cur, n);
    b->nl.count = carve<int>(cur, pbins_cap);
    b->nl.start = carve<int>(cur, pbins_cap + 1);
    b->nl.tmp = carve<int>(cur, pbins_cap / 1024 + 2);
    b->nl.xyzq = carve<double4>(cur, nl_cap);
    b->nl.xyzf = carve<float4>(cur, nl_cap);
    b->nl.sp = carve<int>(cur, nl_cap);
    b->nl.cap = nl_cap;
    b->nl.bins_cap = pbins_cap;
    b->pbin_xblocks = b->lay[DISCOS_LB].pbin_xblocks;
    b->pbin_off = carve<int>(cur, count + 1);
    b->sid = carve<int>(cur, n);
    b->ssp = carve<int>(cur, n);
    b->perm = carve<int>(cur, n);
    b->ion_bin = carve<int>(cur, n);
    b->ion_rank = carve<int>(cur, n);
    b->ion_rep = carve<int>(cur, n);
    b->bin_count = carve<int>(cur, nbins_cap);
    b->bin_start = carve<int>(cur, nbins_cap + 1);
    b->scan_tmp = carve<int>(cur, nblk);
    b->rho = carve<double>(cur, b->ncell_tot);
    b->phi = carve<double>(cur, b->ncell_tot);
    b->spec = carve<double2>(cur, b->nspec_tot);
    b->cprime = carve<double>(cur, ncp);
    b->zg = carve<double>(cur, std::max<int64_t>(zg_len, 1));
    for (int v = 0; v < 3; ++v) {
        b->ztasks[v] = carve<int2>(cur, std::max<size_t>(zt[v].size(), 1));
        b->ztasks_n[v] = (int)zt[v].size();
    }
    b->fp = carve<double>(cur, 3 * n);
    b->flags = carve<int>(cur, 64);
    b->step_d = carve<uint64_t>(cur, 1);
    b->mode_off = carve<int>(cur, count + 1);
    b->mode_rep = carve<int>(cur, count);
    b->reps_d = carve<discos::RepDev>(cur, count);
    for (int kind = 0; kind < 2; ++kind)
        for (int v = 0; v < 2; ++v) {
            b->tasks[kind][v] = carve<int2>(cur, std::max<size_t>(tk[kind][v].size(), 1));
            b->ntasks[kind][v] = (int)tk[kind][v].size();
        }
    b->walls = carve<double>(cur, std::max<int64_t>(wall, 1));
    double2* tw_d = carve<double2>(cur, tw_all.size());
    for (size_t c = 0; c < b->classes.size(); ++c) {
        b->classes[c].tw_x = tw_d + tw_at[c].first;
        b->classes[c].tw_y = tw_d + tw_at[c].second;
    }
    b->idirect = carve<int>(cur, count);
    b->sdirect = carve<int>(cur, count);
    for (int r = 0; r < count; ++r)
        b->ions_per_tile.push_back(2048.0 * reps[r].n / ((double)reps[r].nx * reps[r].ny * reps[r].nz));
    // the batched FFT passes' class table (block ranges and LDS as the per-grid passes)
    b->fcls = carve<discos::FftClassDev>(cur, b->classes.size());
    std::vector<discos::FftClassDev> fcls;
    b->fft_xblocks = b->fft_yblocks = 0;
    b->fft_xlds = b->fft_ylds = 0;
    for (const discos::BatchClass& k : b->classes) {
        discos::FftClassDev f{};
        f.tw_x = k.tw_x;
        f.tw_y = k.tw_y;
        f.cell_off = k.cell_off;
        f.spec_off = k.spec_off;
        f.nx = k.nx;
        f.ny = k.ny;
        f.nxh = k.nx / 2 + 1;
        f.logx = __builtin_ctz((unsigned)k.nx);
        f.logy = __builtin_ctz((unsigned)k.ny);
        f.npairs = k.rows / 2;
        f.ppb = std::max(1, 2048 / k.nx);
        f.xb0 = b->fft_xblocks;
        f.ltpb = __builtin_ctz((unsigned)std::max(1, 1024 / k.ny));
        f.ncol = f.nxh * k.levels;
        f.yb0 = b->fft_yblocks;
        b->fft_xblocks += (f.npairs + f.ppb - 1) / f.ppb;
        b->fft_yblocks += (f.ncol + (1 << f.ltpb) - 1) >> f.ltpb;
        b->fft_xlds = std::max(b->fft_xlds, (size_t)f.ppb * k.nx * sizeof(double2));
        b->fft_ylds = std::max(b->fft_ylds, ((size_t)k.ny << f.ltpb) * sizeof(double2));
        fcls.push_back(f);
    }
    // host tables -> device
    std::vector<int> ion_rep(n, 0);
    std::vector<double> walls(std::max<int64_t>(wall, 1), 0.0);
    for (int r = 0; r < count; ++r) {
        for (int64_t i = b->ion_off[r]; i < b->ion_off[r + 1]; ++i) ion_rep[i] = r;
        discos::RepDev& d = b->reps_h[r];
        const int64_t w0 = reinterpret_cast<int64_t>(d.w.value[0]);
        const int64_t ncol = (int64_t)reps[r].nx * reps[r].ny;
        for (int64_t k = 0; k < ncol; ++k) {
            walls[w0 + k] = reps[r].bc_value[0];
            walls[w0 + ncol + k] = reps[r].bc_value[1];
        }
        d.w.value[0] = b->walls + w0;
        d.w.value[1] = b->walls + w0 + ncol;
    }
    bool ok = hipMemcpy(b->ion_rep, ion_rep.data(), n * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->walls, walls.data(), walls.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->reps_d, b->reps_h.data(), count * sizeof(discos::RepDev), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->pbin_off, pbin_off.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->mode_off, mode_off.data(), (count + 1) * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->mode_rep, mode_rep.data(), count * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(tw_d, tw_all.data(), tw_all.size() * sizeof(double2), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->fcls, fcls.data(), fcls.size() * sizeof(discos::FftClassDev),
                         hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && set_direct(b, 0, b->cfg.interp_direct) && set_direct(b, 1, b->cfg.spread_direct);
    for (int kind = 0; kind < 2; ++kind)
        for (int v = 0; v < 2; ++v)
            if (!tk[kind][v].empty())
                ok = ok && hipMemcpy(b->tasks[kind][v], tk[kind][v].data(), tk[kind][v].size() * sizeof(int2),
                                     hipMemcpyHostToDevice) == hipSuccess;
    for (int v = 0; v < 3; ++v)
        if (!zt[v].empty())
            ok = ok && hipMemcpy(b->ztasks[v], zt[v].data(), zt[v].size() * sizeof(int2),
                                 hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && discos::batch_pivots(b, 0) == DISCOS_OK && hipStreamSynchronize(0) == hipSuccess;
    ok = ok && hipMemset(b->flags, 0, 64 * sizeof(int)) == hipSuccess;
    // bin counts start at zero; the scan that reads them clears them again
    ok = ok && hipMemset(b->bin_count, 0, nbins_cap * sizeof(int)) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        destroy(b);
        return DISCOS_E_HIP;
    }
    *out = b;
    return DISCOS_OK;
}

int discos_batch_destroy(discos_batch* b) {
    if (!b) return DISCOS_E_ARG;
    const bool synced = hipDeviceSynchronize() == hipSuccess;
    return destroy(b) && synced ? DISCOS_OK : DISCOS_E_HIP;
}

int discos_batch_step(discos_batch* b, double* pos, double* q, int32_t* id, int32_t* species,
                      uint64_t step, uint32_t flags, void* stream) {
    if (!b) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    b->last_stream = s;
    if (flags & ~DISCOS_BATCH_GRAPH) return fail(b, DISCOS_E_ARG, "unknown batch step flags");
    if (b->n_tot > 0 && (!pos || !q || !id || !species)) return fail(b, DISCOS_E_ARG, "null ion array");
    if (!(flags & DISCOS_BATCH_GRAPH)) {
        int rc = discos::batch_set_step(b, step, s);
        if (!rc) rc = run_step(b, pos, q, id, species, s);
        b->next_step = ~uint64_t(0);  // the device counter no longer matches a graph's view
        return rc ? fail(b, rc, "batch step launch failed") : DISCOS_OK;
    }
    const void* args[4] = {pos, q, id, species};
    const bool same = b->exec && args[0] == b->graph_args[0] && args[1] == b->graph_args[1] &&
                      args[2] == b->graph_args[2] && args[3] == b->graph_args[3];
    if (!same) {
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        if (b->graph) {
            (void)hipGraphDestroy(b->graph);
            b->graph = nullptr;
        }
        if (hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(b, DISCOS_E_HIP, "graph capture could not start");
        const int rc = run_step(b, pos, q, id, species, b->own);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->own, &g);
        if (rc || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return fail(b, DISCOS_E_HIP, "graph capture failed");
        }
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
            b->exec = nullptr;
            return fail(b, DISCOS_E_HIP, "graph instantiation failed");
        }
        for (int k = 0; k < 4; ++k) b->graph_args[k] = args[k];
        b->next_step = ~uint64_t(0);
    }
    // the graph was captured on the batch's own stream; it replays on the caller's, in
    // order with the caller's other work and without cross-stream events
    if (step != b->next_step && discos::batch_set_step(b, step, s))
        return fail(b, DISCOS_E_HIP, "step counter update failed");
    if (hipGraphLaunch(b->exec, s) != hipSuccess) return fail(b, DISCOS_E_HIP, "graph launch failed");
    b->next_step = step + 1;
    return DISCOS_OK;
}

int discos_batch_tune(discos_batch* b, const double* pos, const double* q, const int32_t* id,
                      const int32_t* species, int32_t* cfg_out, void* stream) {
    if (!b) return DISCOS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    b->last_stream = s;
    if (b->n_tot > 0 && (!pos || !q || !id || !species)) return fail(b, DISCOS_E_ARG, "null ion array");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(b, DISCOS_E_HIP, "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(b, DISCOS_E_HIP, "event create");
    }
    const int reps = 3;
    bool timing_ok = true;  // a failed event call times a candidate as never best
    auto timed = [&](auto&& fn) -> float {
        fn();  // warm
        bool ok = hipEventRecord(e0, s) == hipSuccess;
        for (int k = 0; k < reps; ++k) fn();
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        timing_ok = timing_ok && ok;
        return ok ? ms : 1e30f;
    };
    // every stage's choices for one bin edge; returns the summed best times of the stages
    // the bin edge affects (cell list, spread, interpolation, near field)
    auto tune_stages = [&](discos::BatchCfg& c, int& rc) -> float {
        const float t_cells = timed([&] {
            discos::batch_cell_list(b, pos, q, const_cast<int*>(id), const_cast<int*>(species), s);
        });
        rc = discos::batch_cell_list(b, pos, q, const_cast<int*>(id), const_cast<int*>(species), s);
        const int blocks[3] = {0, 4 * b->ncu, 8 * b->ncu};
        // spread: tile edge x persistent blocks
        float best = 1e30f;
        c = b->cfg;
        for (int t : {8, 16})
            for (int nb : blocks) {
                b->cfg.spread_t = t;
                b->cfg.spread_blocks = nb;
                const float ms = timed([&] { discos::batch_spread(b, s); });
                if (ms < best) {
                    best = ms;
                    c.spread_t = t;
                    c.spread_blocks = nb;
                }
            }
        b->cfg.spread_t = c.spread_t;
        b->cfg.spread_blocks = c.spread_blocks;
        // spread: the density below which channels add their ions with global atomics
        best = 1e30f;
        for (int th : {0, 8, 24, 64, 1 << 30}) {
            if (!set_direct(b, 1, th)) {
                timing_ok = false;
                break;
            }
            const float ms = timed([&] { discos::batch_spread(b, s); });
            if (ms < best) {
                best = ms;
                c.spread_direct = th;
            }
        }
        const float t_spread = best;
        if (!set_direct(b, 1, c.spread_direct)) timing_ok = false;
        if (!rc) rc = discos::batch_spread(b, s);
        if (!rc) rc = discos::batch_poisson(b, s);
        // interpolation: tile shape x persistent blocks
        best = 1e30f;
        for (int t : {8, 16})
            for (int nb : blocks) {
                b->cfg.interp_t = t;
                b->cfg.interp_blocks = nb;
                const float ms = timed([&] { discos::batch_interp(b, s); });
                if (ms < best) {
                    best = ms;
                    c.interp_t = t;
                    c.interp_blocks = nb;
                }
            }
        b->cfg.interp_t = c.interp_t;
        b->cfg.interp_blocks = c.interp_blocks;
        // interpolation: the density below which channels skip the staged tiles
        best = 1e30f;
        for (int th : {0, 8, 24, 64, 1 << 30}) {
            if (!set_direct(b, 0, th)) {
                timing_ok = false;
                break;
            }
            const float ms = timed([&] { discos::batch_interp(b, s); });
            if (ms < best) {
                best = ms;
                c.interp_direct = th;
            }
        }
        const float t_interp = best;
        if (!set_direct(b, 0, c.interp_direct)) timing_ok = false;
        // per-ion stages: workgroup size (the padded list and the near-field pass)
        best = 1e30f;
        for (int wg : {64, 128, 256}) {
            b->cfg.ion_block = wg;
            const float ms = timed([&] { discos::batch_near(b, s); });
            if (ms < best) {
                best = ms;
                c.ion_block = wg;
            }
        }
        b->cfg = c;
        return t_cells + t_spread + t_interp + best;
    };
    // the bin edge: 2 cells, and 4 cells where every channel is wide enough for it
    int rc = 0;
    discos::BatchCfg c = b->cfg;
    float best_total = 1e30f;
    float totals[3] = {0.0f, 0.0f, 0.0f};
    for (int lb = 1; lb <= 2 && !rc; ++lb) {
        if (!b->lay[lb].ok) continue;
        if (!apply_layout(b, lb)) {
            timing_ok = false;
            break;
        }
        discos::BatchCfg cl;
        const float total = tune_stages(cl, rc);
        totals[lb] = total;
        if (total < best_total) {
            best_total = total;
            c = cl;
        }
    }
    if (!apply_layout(b, c.lb)) timing_ok = false;
    if (!set_direct(b, 0, c.interp_direct) || !set_direct(b, 1, c.spread_direct)) timing_ok = false;
    b->cfg = c;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // a captured graph holds the previous launch shapes
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    if (cfg_out) {
        cfg_out[0] = c.spread_t;
        cfg_out[1] = c.spread_blocks;
        cfg_out[2] = c.interp_t;
        cfg_out[3] = c.interp_blocks;
        cfg_out[4] = c.ion_block;
        cfg_out[5] = c.interp_direct;
        cfg_out[6] = c.spread_direct;
        cfg_out[7] = 1 << c.lb;
        // microseconds of one pass of the bin-dependent stages, per bin edge (0: not tried)
        cfg_out[8] = (int32_t)(1e3f * totals[1] / reps + 0.5f);
        cfg_out[9] = (int32_t)(1e3f * totals[2] / reps + 0.5f);
    }
    if (rc || !timing_ok || hipGetLastError() != hipSuccess)
        return fail(b, DISCOS_E_HIP, "tuning launch failed");
    return DISCOS_OK;
}

int discos_batch_set_bin(discos_batch* b, int32_t bin) {
    if (!b) return DISCOS_E_ARG;
    if (bin != 2 && bin != 4) return fail(b, DISCOS_E_ARG, "bin edge must be 2 or 4 cells");
    const int lb = bin == 2 ? 1 : 2;
    if (!b->lay[lb].ok) return fail(b, DISCOS_E_SHAPE, "a channel is too narrow for this bin edge");
    if (!apply_layout(b, lb)) return fail(b, DISCOS_E_HIP, "bin layout update failed");
    return DISCOS_OK;
}

int discos_batch_check(discos_batch* b) {
    if (!b) return DISCOS_E_ARG;
    if (hipStreamSynchronize(b->last_stream) != hipSuccess || hipStreamSynchronize(b->own) != hipSuccess)
        return fail(b, DISCOS_E_HIP, "sync failed");
    int f = 0;
    if (hipMemcpy(&f, b->flags, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(b, DISCOS_E_HIP, "flag read failed");
    if (f && hipMemset(b->flags, 0, sizeof(int)) != hipSuccess)
        return fail(b, DISCOS_E_HIP, "flag reset failed");
    if (f & DISCOS_FLAG_NONFINITE) return fail(b, DISCOS_E_NONFINITE, "non-finite position");
    if (f & DISCOS_FLAG_BAD_SPECIES) return fail(b, DISCOS_E_ARG, "species index out of range");
    if (f & DISCOS_FLAG_CAPACITY) return fail(b, DISCOS_E_CAPACITY, "tile candidate rows exceeded");
    if (f & DISCOS_FLAG_NOT_NEUTRAL) return fail(b, DISCOS_E_NOT_NEUTRAL, "channel not neutral");
    if (f & DISCOS_FLAG_OUT_OF_DOMAIN) return fail(b, DISCOS_E_OUT_OF_DOMAIN, "ion outside its channel");
    return DISCOS_OK;
}

const char* discos_batch_last_error(discos_batch* b) {
    if (!b) return "null batch";
    return b->err.c_str();
}

}  // extern "C"
