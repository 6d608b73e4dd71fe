// Host-side view of the context and the launchers shared by the kernel files.
#pragma once

#include <algorithm>
#include <string>
#include <array>
#include <vector>

#include "common.h"

namespace discos {

// The near-field pass's own copy of the cell list, padded so that every search row is
// one contiguous run: R ghost bins on each x and y side hold the periodic copies (x and y
// shifted by a period), and R ghost slabs beyond each wall hold the mirror images of the
// first R slabs (z mirrored, charge times the wall's image sign, species -1).
struct NearList {
    int* count;      // [bins_cap] entries per padded bin
    int* start;      // [bins_cap + 1] exclusive starts (start[nb] = total)
    int* tmp;        // scan block sums
    double4* xyzq;   // [cap] x, y, z, q of every copy
    float4* xyzf;    // [cap] the same in FP32 (the candidate filter)
    int* sp;         // [cap] species of the copy, -1 for wall images
    int64_t cap, bins_cap;
};

struct Ctx {
    discos_grid grid;
    GridDev gd;
    int64_t n_max;
    int device;
    int64_t ncell;   // nx ny nz
    int64_t nface_z; // nx ny (nz + 1)
    int64_t nmode;   // (nx/2 + 1) ny
    int64_t nbins;
    // sorted ion copies (cell-list order): (x, y, z, q) with x, y reduced into
    // [0, L], plus ids, species and the permutation back to caller order
    double4* sxyzq;
    int *sid, *ssp, *perm;
    int *ion_bin, *ion_rank;
    int *bin_count, *bin_start, *scan_tmp;
    // grid work arrays
    double *rho, *phi;
    double2* spec;   // half spectrum [nz][ny][nx/2+1]
    double* cprime;  // z-solve pivots [nz][nmode] (or Thomas scratch when nz > 128)
    int zg_key;      // wall types the pivots in cprime were computed for (-1: none)
    double* fp;      // [3][n_max] per-ion forces in cell-list order
    double* fnear;   // [3][n_max] near-field forces of a dry step computed beside the grid stages
    hipStream_t side = nullptr;                      // the near field's stream in a dry step
    int serial = 0;                                  // DISCOS_CREATE_SERIAL: no side stream work
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;  // the cell list is built / the pass is done
    double2 *tw_x, *tw_y;
    NearList nl;     // the near-field pass's padded copy of the cell list
    // walls of mixed type (a capacitance solve on the wall layers): pcg, [2][ncell], the
    // right-hand side and solution of the second uniform-wall solve; cap, the per-mode
    // wall Green's function and preconditioner ([3][ny][nx/2+1] each, for the reference
    // pair cap_key) and six vectors on the two wall planes ([2][ny][nx] each); pcg_s, the
    // iteration's scalars; wm_*: the wall maps of the current call (read on the host)
    double* pcg;
    double* cap;
    int cap_key;     // reference pair and walls with unknowns the tables hold (-1: none)
    double cap_eps;  // and the permittivity they were scaled with
    double* pcg_s;
    int wm_mixed;
    int mx_iters;  // iterations of the last mixed-wall solve
    int wm_ref[2];
    // walls of mixed type solved directly: the inverse of -S on the cap_nd unknowns
    // (column-major, symmetric), their wall-plane indices and two packed vectors,
    // allocated for cap_alloc unknowns when a map set is first solved this way
    int mx_iterative;  // DISCOS_CREATE_MIXED_ITERATIVE: conjugate gradients only
    double* cap_inv;
    int* cap_idx;
    double* cap_vec;
    int64_t cap_alloc;
    int cap_nd;         // unknowns of the held inverse (-1: none, 0: solve iteratively)
    int cap_dkey;       // table key, generation of the maps' contents and permittivity
    uint64_t cap_dgen;  // the held inverse belongs to
    double cap_deps;
    uint64_t wm_gen;    // advances whenever the wall maps' contents change
    std::vector<int32_t> wm_host[2];
    void* rb;           // rocBLAS handle of the factorisation (created on first use)
    // hydrodynamics (allocated with DISCOS_CREATE_HYDRO)
    int hydro;
    double2* hspec;   // spectra of u, v, w, p: nz, nz, nz+1, nz levels of [ny][nx/2+1]
    double* hfac;     // block-Thomas factors of the Stokes mode systems, 14 doubles per level and mode
    int hfac_key;     // wall types hfac was computed for: bit 0 lower slip, bit 1 upper slip
    double* hz_diag;  // stress normals: xx, yy, zz, xy per cell
    double* hz_edge;  // stress normals: xz, yz per z-level edge
    double* hvel;     // face velocity scratch for the wet step (3 face arrays)
    double* hfor;     // face force scratch (3 face arrays)
    double* hvi;      // [3][n_max] interpolated ion velocities
    double* part;     // [3][PART_MAX] partial sums of the deterministic reductions (the third:
                      // sum w(z) q of the last energy / flux forward pass)
    double* bcg;      // [2][ny][nx] wall-field adjoints gathered from the ghost layers
    // hydrodynamic kernel per species: [DISCOS_HY_MAXSP + 1][4] rows (w, beta, 1 / alpha,
    // 1 / integral), w = 0 for the 4-point Peskin kernel (every row past the set ones,
    // and the extra last row that species out of range read);
    // hy_km: half-width of the node window of the widest set kernel (0: all Peskin)
    double* hy_tab;
    int hy_km;
    int* flags;
    void* pool;
    void* hpool;
    size_t pool_bytes;
    hipStream_t last_stream;
    std::string err;
    // cell-list generations: every build advances cl_gen; discos_energy_flux records the
    // generation and ion count of the list it built (for the backward pass to reuse)
    uint64_t cl_gen;
    uint64_t ef_gen;
    int ef_n;
    double ef_wq;  // flux weight (1 / (2 eta nz)) the held sum w q was taken with; 0: none
    // stage timing (discos_profile): one row of DISCOS_NSTAGE + 1 events per step,
    // for up to PROF_MAX steps
    int profile;
    uint32_t prof_stages;  // stages timed (bit k: stage k)
    uint32_t prof_marks;   // events recorded: both bounds of every timed stage
    int prof_steps;
    hipEvent_t* ev;
    // a dry step whose near field ran on the side stream: the event that opened its
    // padded-list stage there (one per profiled step), and which steps did
    hipEvent_t* ev_side = nullptr;
    std::vector<char> prof_side;
};

#define PROF_MAX 512

// A batch of independent channels (one dry step each per discos_batch_step).
struct BatchClass {   // channels of one (nx, ny): their grids and spectra are contiguous
    int nx, ny, rep_first, rep_count;
    int64_t cell_off, spec_off;  // of the first channel of the class
    int rows, levels;            // sum of ny nz and of nz over the class
    double2 *tw_x, *tw_y;
};

// One (nx, ny) class as the batched FFT passes read it: its first x-pass block (xb0,
// blocks of ppb row pairs) and first y-pass block (yb0, blocks of 2^ltpb of its ncol
// spectrum columns).
struct FftClassDev {
    const double2* tw_x;
    const double2* tw_y;
    int64_t cell_off, spec_off;
    int nx, ny, nxh, logx, logy;
    int npairs, ppb, xb0;
    int ltpb, ncol, yb0;
};

struct BatchCfg {   // launch choices (the autotuner's output)
    int spread_t;       // spread tile edge: 8 or 16
    int spread_blocks;  // persistent blocks of the spread (0: one per task)
    int interp_t;       // interpolation tile: 16 -> 16x16x8, 8 -> 8x8x8
    int interp_blocks;  // persistent blocks of the interpolation (0: one per task)
    int ion_block;      // workgroup size of the per-ion kernels
    int interp_direct;  // channels with fewer ions per 2048 cells are interpolated one
                        // thread per ion instead of by staged tiles
    int spread_direct;  // likewise spread one thread per ion with global atomics
    int lb;             // log2 of the cell-list bin edge in cells (1: 2 cells, 2: 4 cells)
};

// The cell list's bins and the near field's padded bins of a batch for one bin edge.
struct BinLayout {
    bool ok = false;            // every channel is wide enough for the search window
    int R = 0;                  // near-field search radius in bins
    int64_t nbins = 0, pbins = 0, nl_entries = 0;
    int pbin_xblocks = 1;       // x blocks of the padded-bin count (the largest channel's)
    std::vector<int> bin_off, pbin_off;  // [channels + 1]
};

struct Batch {
    int R;
    double h;
    discos_params p;              // shared physics (copied)
    std::vector<discos_replica> reps;
    std::vector<RepDev> reps_h;
    RepDev* reps_d;
    int64_t n_tot, ncell_tot, nspec_tot, nbins_tot;
    std::vector<int64_t> ion_off;  // [R + 1]
    int* ion_rep;                  // [n_tot] channel of each ion slot
    int* mode_off;                 // [R + 1] prefix of the channels' mode counts (class order)
    int* mode_rep;                 // [R] channel of each position in mode_off
    int64_t nmode_tot;
    int2* tasks[2][2];             // [kernel: spread, interp][variant]: (channel, tile)
    int ntasks[2][2];
    int2* ztasks[3];               // z-solve with pivots, L = 8, 16, 32: (channel, first mode)
    int ztasks_n[3];
    std::vector<std::array<int64_t, 4>> zshapes;  // (nx, ny, nz, pivot offset) per grid shape
    double* zg;                    // pivots of every shape, [nz][nmode] each
    bool z_legacy = false;         // some channel has nz > 128 (per-mode Thomas, scratch cprime)
    bool z_singular = false;       // both walls Neumann
    std::vector<BatchClass> classes;
    int* idirect;                 // [channels] 1: interpolated one thread per ion
    int n_direct;                 // channels so flagged
    int* sdirect;                 // [channels] 1: spread one thread per ion
    int n_sdirect;
    std::vector<double> ions_per_tile;  // per channel: ions per 2048 cells
    FftClassDev* fcls;            // [classes] for the batched FFT passes
    int fft_xblocks, fft_yblocks; // blocks of the x passes and of the y pass
    size_t fft_xlds, fft_ylds;    // their dynamic LDS
    double* walls;                 // per-channel wall fields [2][ny][nx], back to back
    double4* sxyzq;
    int *sid, *ssp, *perm, *ion_bin, *ion_rank, *bin_count, *bin_start, *scan_tmp;
    NearList nl;                   // padded copy of the near field (every channel's bins)
    int* pbin_off;                 // [R + 1] first padded bin of each channel (device)
    int pbin_xblocks;  // x blocks of the per-channel padded-bin grid (the largest channel's)
    int64_t pbins_tot;             // padded bins of the current bin edge
    BinLayout lay[3];              // by log2 of the bin edge (entries 1 and 2)
    double *rho, *phi, *cprime, *fp;
    double2* spec;
    int* flags;
    uint64_t* step_d;
    void* pool;
    BatchCfg cfg;
    int ncu;
    hipStream_t own;               // stream the graph is captured on (it replays on the caller's)
    hipGraph_t graph;
    hipGraphExec_t exec;
    const void* graph_args[4];
    uint64_t next_step;
    hipStream_t last_stream;
    std::string err;
};
#define PART_MAX 1024

// Record the event that closes stage k of the current profiled step.
inline void stage_mark(Ctx* c, int k, hipStream_t s) {
    if (c->profile && c->prof_steps < PROF_MAX && ((c->prof_marks >> k) & 1u))
        // a failed record surfaces when discos_profile_read queries the event
        (void)hipEventRecord(c->ev[(size_t)c->prof_steps * (DISCOS_NSTAGE + 1) + k], s);
}

// Record the opening of stage k (the padded list) on the side stream s of the current
// profiled step, whose closing and the earlier stages' events are recorded elsewhere.
inline void stage_open_side(Ctx* c, int k, hipStream_t s) {
    if (c->profile && c->prof_steps < PROF_MAX && ((c->prof_marks >> k) & 1u)) {
        (void)hipEventRecord(c->ev_side[c->prof_steps], s);
        c->prof_side[c->prof_steps] = 1;
    }
}

WallDev wall_of(const discos_params* p);

// Cell list from positions (and optional companions) in caller order.
int build_cell_list(Ctx* c, int n, const double* x, const double* y, const double* z,
                    const double* q, const int* id, const int* sp, hipStream_t s,
                    const double* w3 = nullptr, int64_t w3_stride = 0);
void fill_f64(double* a, int64_t n, double v, hipStream_t s);
// Exclusive scan of count[0, nb) into start[0, nb] (start[nb] = total), clearing count.
void scan_counts(int* count, int64_t nb, int* tmp, int* start, hipStream_t s);
// Padded near-field list sizes for a grid: entries for n ions and padded bins, for search
// radii up to 3 bins.
int64_t near_list_entries(const GridDev& g, int64_t n);
int64_t near_list_bins(const GridDev& g, int R);

// S^es over the cell list: rho = S q (sorted copies sx..sq) with fold signs; optional
// wall terms of the discrete Poisson problem.
int spread_charge_sorted(Ctx* c, const discos_params* p, int add_bc, double* out, hipStream_t s);

// Poisson solve in place capable (rhs may equal phi).  project != 0: the pseudo-inverse
// for any rhs in the all-Neumann case (the adjoint solve), without the neutrality flag.
int solve_poisson(Ctx* c, const double* rhs, const discos_params* p, double* phi, hipStream_t s,
                  int mark_base = -1, int project = 0);

// Poisson solve with walls of mixed type (the uniform pair ref, corrected on the wall
// layers by a capacitance system); returns DISCOS_E_NOT_CONVERGED if the tolerance was
// not reached.
int solve_poisson_mixed(Ctx* c, const double* rhs, const discos_params* p, const int ref[2],
                        double* phi, hipStream_t s);
// out = F^-1 [C_k F in] on a pair of (x, y) planes with per-mode 2 x 2 maps coef.
int plane_pair_filter(Ctx* c, const double* in, double* out, const double* coef, hipStream_t s);

// Frees the dense capacitance inverse and its rocBLAS handle (false on a runtime error).
bool release_dense_capacitance(Ctx* c);

// E^P (op DISCOS_INTERP_E), q (E^P + E_ext) (DISCOS_INTERP_FORCE) or J phi
// (DISCOS_INTERP_PHI) for the ions of the cell list; out[perm[i]] if scatter, else out[i].
int interp_es_sorted(Ctx* c, int op, int n, const double* phi, const discos_params* p,
                     double* out, int64_t out_stride, int scatter, hipStream_t s);

// Caller arrays of a dry step whose update the force pass performs itself.
struct DryStepOut {
    uint64_t step;
    double* pos;
    double* q;
    int* id;
    int* sp;
};

// Near-field + wall (+ LJ) forces over the cell list; out[perm] += F if scatter, else
// out[sorted] += F.  mark >= 0: profiling stage mark between the list build and the
// force pass.  upd: a dry step's update from the complete forces out[sorted] + F is
// done in the same pass (out is not written).
int near_field_sorted(Ctx* c, int n, const discos_params* p, double* out, int64_t out_stride,
                      int scatter_to_caller, hipStream_t s, int mark = -1,
                      const DryStepOut* upd = nullptr, bool store = false);

// Random finite difference of the thermal forcing (scale = kT / delta, half = delta / 2;
// scale 0: off); sid holds the ions' stable ids in cell-list order.
struct RfdDev {
    const int* sid;
    double scale, half;
    uint64_t seed, step;
    const double* w;   // the ions' normals W, [3][wstride] in cell-list order (set by the spread)
    int64_t wstride;
};

// S^hy of the sorted forces c->fp onto the three face arrays of out (+ the thermal
// forcing when rfd is given; n: the ions of the cell list, whose normals it draws).
// species != 0: each ion's kernel from c->hy_tab by its species c->ssp.
int spread_force_sorted(Ctx* c, double* out, hipStream_t s, const RfdDev* rfd = nullptr,
                        int species = 0, int n = 0);
// Factorisation of the Stokes mode systems of the context's grid (once, at creation).
int stokes_factor(Ctx* c, hipStream_t s);
// Stokes solve with no-slip walls (f: three face arrays; vel likewise; pres nullable).
int solve_stokes(Ctx* c, const double* f, const discos_params* p, uint64_t step, int noise,
                 double* vel, double* pres, hipStream_t s);
// J^hy of the face velocity for the ions of the cell list.
int interp_hy_sorted(Ctx* c, int n, const double* vel, double* out, int64_t stride, int scatter,
                     hipStream_t s, int species = 0);

// The wet step's midpoint velocities c->hvi = J(x*) v, x* = x + dt/2 J(x) v.
int midpoint_velocity(Ctx* c, int n, const double* vel, double dt, hipStream_t s, int species = 0);

// Update of the sorted ions from their complete forces c->fp (dry terms of eq step2)
// plus dt * vwet (nullable, [3][n_max] sorted), written to the caller's arrays in
// cell-list order.
int update_sorted(Ctx* c, int n, const discos_params* p, uint64_t step, const double* vwet,
                  double* pos, double* q, int* id, int* sp, hipStream_t s,
                  const double* fp2 = nullptr);

// U = (1/2) dV <c->rho, phi> and Q = sum w(z) F_x over the sorted forces c->fp into
// out[0], out[1] (device).
int energy_flux(Ctx* c, int n, const discos_params* p, const double* phi, double* out, hipStream_t s);
// Reverse sweep of energy_flux over the current cell list (outputs nullable).
int energy_flux_backward(Ctx* c, int n, const discos_params* p, const double* phi, const double* gvec,
                         double* dpos, double* dq, double* dlo, double* dhi, double* de, bool reuse,
                         hipStream_t s);

// Batched stages (one launch each over all channels of the batch).
int batch_cell_list(Batch* b, const double* pos, const double* q, const int* id, const int* sp,
                    hipStream_t s);
int batch_spread(Batch* b, hipStream_t s);
int batch_pivots(Batch* b, hipStream_t s);
int batch_poisson(Batch* b, hipStream_t s);
int batch_interp(Batch* b, hipStream_t s);
int batch_near(Batch* b, hipStream_t s);
int batch_update(Batch* b, double* pos, double* q, int* id, int* sp, hipStream_t s);
int batch_set_step(Batch* b, uint64_t v, hipStream_t s);
int near_radius_bins_h(double h, const discos_params* p, int lb);

}  // namespace discos
