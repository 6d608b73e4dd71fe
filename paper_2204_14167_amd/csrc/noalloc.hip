// S^es charge spreading without a context and without any allocation: the variant of
// discos_spread(DISCOS_SPREAD_CHARGE) for callers that cannot allocate device memory.
//
// The cell list that the spread reads (bin counts and starts, the sorted ion copies and
// the permutation) lives in one file-scope device array, `scratch`, of a fixed size.
// Host code never names that array as an address: on the first call on a device (with
// that device current) hipGetSymbolAddress gives the device address of that device's
// copy, which is kept per device and is the only pointer the kernels receive.
#include <mutex>

#include "kernels.h"

namespace {

constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr int64_t NA_IONS = DISCOS_NOALLOC_MAX_IONS;
constexpr int64_t NA_BINS = DISCOS_NOALLOC_MAX_BINS;
constexpr int64_t NA_SCAN = NA_BINS / 1024 + 2;

// Layout of the scratch array (each part 256-byte aligned).
constexpr size_t OFF_SXYZQ = 0;
constexpr size_t OFF_PERM = OFF_SXYZQ + al256(NA_IONS * sizeof(double4));
constexpr size_t OFF_BIN = OFF_PERM + al256(NA_IONS * sizeof(int));
constexpr size_t OFF_RANK = OFF_BIN + al256(NA_IONS * sizeof(int));
constexpr size_t OFF_COUNT = OFF_RANK + al256(NA_IONS * sizeof(int));
constexpr size_t OFF_START = OFF_COUNT + al256(NA_BINS * sizeof(int));
constexpr size_t OFF_STMP = OFF_START + al256((NA_BINS + 1) * sizeof(int));
constexpr size_t OFF_FLAGS = OFF_STMP + al256(NA_SCAN * sizeof(int));
constexpr size_t NA_BYTES = OFF_FLAGS + 256;
static_assert(NA_BYTES < ((size_t)8 << 20), "scratch of the no-allocation spread above 8 MiB");

}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

std::mutex na_mutex;
void* na_ptr[64] = {};  // device address of `scratch`, per device ordinal

// The device address of this device's scratch (null on failure).
void* scratch_ptr(int dev) {
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        na_ptr[dev] = p;
    }
    return na_ptr[dev];
}

__global__ void na_clear_kernel(int* __restrict__ count, int64_t nb, int* __restrict__ flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nb;
         i += (int64_t)gridDim.x * blockDim.x)
        count[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) flags[0] = 0;
}

// The sticky device flags of this call as one status code (precedence of discos_check).
__global__ void na_status_kernel(const int* __restrict__ flags, int32_t* __restrict__ status) {
    const int f = flags[0];
    int32_t s = DISCOS_OK;
    if (f & DISCOS_FLAG_NONFINITE)
        s = DISCOS_E_NONFINITE;
    else if (f & DISCOS_FLAG_CAPACITY)
        s = DISCOS_E_CAPACITY;
    else if (f & DISCOS_FLAG_OUT_OF_DOMAIN)
        s = DISCOS_E_OUT_OF_DOMAIN;
    status[0] = s;
}

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

}  // namespace

extern "C" int discos_spread_charge_noalloc(const discos_grid* grid, int64_t n, const double* pos,
                                            const double* q, const discos_params* p,
                                            uint32_t flags, double* rho, int32_t* status,
                                            void* stream) {
    if (!grid || !p || !rho || (n > 0 && (!pos || !q))) return DISCOS_E_ARG;
    if ((flags & ~(uint32_t)DISCOS_SPREAD_ADD_BC) != 0) return DISCOS_E_ARG;
    if (!pow2_in(grid->nx, 8, 1024) || !pow2_in(grid->ny, 8, 1024) || grid->nz < 4 ||
        grid->nz > 8192 || !(std::isfinite(grid->h) && grid->h > 0.0))
        return DISCOS_E_SHAPE;
    if (!(std::isfinite(p->eps) && p->eps > 0.0)) return DISCOS_E_ARG;
    for (int w = 0; w < 2; ++w)
        if ((p->bc_type[w] != DISCOS_BC_DIRICHLET && p->bc_type[w] != DISCOS_BC_NEUMANN) ||
            p->bc_type_map[w] != nullptr)  // walls of one type each only
            return DISCOS_E_ARG;
    discos::Ctx c{};
    discos::GridDev& g = c.gd;
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
    const int64_t nbins = (int64_t)g.nbx * g.nby * g.nbz;
    // sizes beyond the fixed scratch are refused before anything is enqueued
    if (n < 0 || n > NA_IONS || nbins > NA_BINS) return DISCOS_E_CAPACITY;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DISCOS_E_HIP;
    char* base = static_cast<char*>(scratch_ptr(dev));
    if (!base) return DISCOS_E_HIP;
    c.grid = *grid;
    c.n_max = NA_IONS;
    c.device = dev;
    c.ncell = (int64_t)g.nx * g.ny * g.nz;
    c.nbins = nbins;
    c.sxyzq = reinterpret_cast<double4*>(base + OFF_SXYZQ);
    c.perm = reinterpret_cast<int*>(base + OFF_PERM);
    c.ion_bin = reinterpret_cast<int*>(base + OFF_BIN);
    c.ion_rank = reinterpret_cast<int*>(base + OFF_RANK);
    c.bin_count = reinterpret_cast<int*>(base + OFF_COUNT);
    c.bin_start = reinterpret_cast<int*>(base + OFF_START);
    c.scan_tmp = reinterpret_cast<int*>(base + OFF_STMP);
    c.flags = reinterpret_cast<int*>(base + OFF_FLAGS);
    hipStream_t s = (hipStream_t)stream;
    // the previous call's contents remain: the bin counts and the flags start at zero
    na_clear_kernel<<<(int)std::min<int64_t>((nbins + 255) / 256, 1024), 256, 0, s>>>(
        c.bin_count, nbins, c.flags);
    if (hipGetLastError() != hipSuccess) return DISCOS_E_HIP;
    int rc = discos::build_cell_list(&c, (int)n, pos, pos + n, pos + 2 * n, q, nullptr, nullptr, s);
    if (rc) return rc;
    rc = discos::spread_charge_sorted(&c, p, (flags & DISCOS_SPREAD_ADD_BC) ? 1 : 0, rho, s);
    if (rc) return rc;
    if (status) {
        na_status_kernel<<<1, 1, 0, s>>>(c.flags, status);
        if (hipGetLastError() != hipSuccess) return DISCOS_E_HIP;
    }
    return DISCOS_OK;
}
