// Cell list: counting sort of ions into bins of DISCOS_BIN^3 cells (row-major bin
// order, x fastest).  Neighbour sets of the near-field pass (Sec. II.B.1, the set
// Omega_i^E of eq fullElectro) and the tile gathers of the spread are read from it.
#include "kernels.h"

namespace discos {

__global__ void fill_i32_kernel(int* __restrict__ a, int64_t n, int v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void fill_f64_kernel(double* __restrict__ a, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// Bin of ion i (bins of its channel start at bin_off) and its rank inside the bin.
// Ions of consecutive lanes that share a bin (the ions of a step arrive in the previous
// step's cell order, so most neighbours in a bin are adjacent) take their ranks from one
// atomic of the first lane of their run: rank = the run's base + the lane's place in it.
// The ranks of a bin are distinct and cover 0 .. count - 1 whatever the arrival order.
// Every lane of the wavefront calls this (active = false for lanes past the last ion).
__device__ __forceinline__ void bin_count_one(const GridDev& g, int bin_off, int i, bool active,
                                              const double* __restrict__ x,
                                              const double* __restrict__ y,
                                              const double* __restrict__ z,
                                              int* __restrict__ count, int* __restrict__ ion_bin,
                                              int* __restrict__ ion_rank, int* __restrict__ flags) {
    int b = -1;
    if (active) {
        const double xi = x[i], yi = y[i], zi = z[i];
        if (!pos_ok(g, xi, yi, zi))
            set_flag(flags, (isfinite(xi) && isfinite(yi) && isfinite(zi))
                                ? DISCOS_FLAG_OUT_OF_DOMAIN
                                : DISCOS_FLAG_NONFINITE);
        int bx, by, bz;
        b = bin_off + ((isfinite(xi) && isfinite(yi) && isfinite(zi) && fabs(xi) < 1e12 * g.h &&
                        fabs(yi) < 1e12 * g.h)
                           ? bin_of(g, xi, yi, zi, bx, by, bz)
                           : 0);
    }
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(b, 1, 64);
    const bool head = active && (lane == 0 || prev != b);
    const unsigned long long heads = __ballot(head);
    const unsigned long long live = __ballot(active);
    // first lane of this lane's run, and the run's length (up to the next head or the last
    // active lane)
    const unsigned long long upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1));
    const int h = active ? 63 - __clzll(upto) : 0;
    const unsigned long long above = heads & ~((2ull << h) - 1) & (h == 63 ? 0ull : ~0ull);
    const int end = above ? __ffsll(above) - 1 : 64 - __clzll(live);
    int base = 0;
    if (head) base = atomicAdd(&count[b], end - h);
    base = __shfl(base, h, 64);
    if (active) {
        ion_bin[i] = b;
        ion_rank[i] = base + (lane - h);
    }
}

__global__ void bin_count_kernel(GridDev g, int n, const double* __restrict__ x,
                                 const double* __restrict__ y, const double* __restrict__ z,
                                 int* __restrict__ count, int* __restrict__ ion_bin,
                                 int* __restrict__ ion_rank, int* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bin_count_one(g, 0, i, i < n, x, y, z, count, ion_bin, ion_rank, flags);
}

__global__ void bin_count_batch_kernel(const RepDev* __restrict__ reps, const int* __restrict__ ion_rep,
                                       int n, const double* __restrict__ x,
                                       const double* __restrict__ y, const double* __restrict__ z,
                                       int* __restrict__ count, int* __restrict__ ion_bin,
                                       int* __restrict__ ion_rank, int* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < n;
    const int r = active ? ion_rep[i] : 0;
    bin_count_one(reps[r].g, reps[r].bin_off, i, active, x, y, z, count, ion_bin, ion_rank, flags);
}

// Exclusive scan of `count` (nb entries) into `start` (nb + 1 entries) in two launches:
// per-block sums, then each block adds the sums of the blocks before it and scans.
#define SCAN_BLOCK 256
#define SCAN_ITEMS 4
#define SCAN_TILE (SCAN_BLOCK * SCAN_ITEMS)

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int& total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        const int a = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[SCAN_BLOCK - 1];
    const int incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ void scan_reduce_kernel(const int* __restrict__ count, int64_t nb,
                                   int* __restrict__ block_sum) {
    __shared__ int sh[SCAN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        if (i < nb) s += count[i];
    }
    int total;
    block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0) block_sum[blockIdx.x] = total;
}

// Also clears the counts it has read, so that the next binning starts from zero
// without a fill (contexts and batches clear them once at creation).  start[nb] receives
// the total.
__global__ void scan_final_kernel(int* __restrict__ count, int64_t nb,
                                  const int* __restrict__ block_sum, int* __restrict__ start) {
    __shared__ int sh[SCAN_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    // this block's offset: the sums of the blocks before it
    int part = 0;
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += SCAN_BLOCK) part += block_sum[j];
    int block_off;
    block_exclusive_scan(part, sh, block_off);
    int v[SCAN_ITEMS];
    int s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        v[k] = (i < nb) ? count[i] : 0;
        if (i < nb) count[i] = 0;
        s += v[k];
    }
    int total;
    int ex = block_exclusive_scan(s, sh, total) + block_off;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + (int64_t)threadIdx.x * SCAN_ITEMS + k;
        if (i < nb) start[i] = ex;
        ex += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BLOCK - 1) start[nb] = ex;
}

void scan_counts(int* count, int64_t nb, int* tmp, int* start, hipStream_t s) {
    const int nblk = (int)((nb + SCAN_TILE - 1) / SCAN_TILE);
    scan_reduce_kernel<<<nblk, SCAN_BLOCK, 0, s>>>(count, nb, tmp);
    scan_final_kernel<<<nblk, SCAN_BLOCK, 0, s>>>(count, nb, tmp, start);
}

// Sorted copies of the ion arrays; perm[sorted] = original index.
__global__ void bin_scatter_batch_kernel(const RepDev* __restrict__ reps,
                                         const int* __restrict__ ion_rep, int n,
                                         const int* __restrict__ ion_bin,
                                         const int* __restrict__ ion_rank,
                                         const int* __restrict__ start, const double* __restrict__ x,
                                         const double* __restrict__ y, const double* __restrict__ z,
                                         const double* __restrict__ q, const int* __restrict__ id,
                                         const int* __restrict__ sp, double4* __restrict__ sxyzq,
                                         int* __restrict__ sid, int* __restrict__ ssp,
                                         int* __restrict__ perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const GridDev& g = reps[ion_rep[i]].g;
    const int d = start[ion_bin[i]] + ion_rank[i];
    if (d < 0 || d >= n) return;  // ranks are a permutation of each bin's slots
    double xi = x[i], yi = y[i];
    if (isfinite(xi) && isfinite(yi)) {
        xi = reduce_periodic(xi, g.Lx);
        yi = reduce_periodic(yi, g.Ly);
    }
    sxyzq[d] = make_double4(xi, yi, z[i], q[i]);
    sid[d] = id[i];
    ssp[d] = sp[i];
    perm[d] = i;
}

__global__ void bin_scatter_kernel(int n, const int* __restrict__ ion_bin,
                                   const int* __restrict__ ion_rank, const int* __restrict__ start,
                                   const double* __restrict__ x, const double* __restrict__ y,
                                   const double* __restrict__ z, const double* __restrict__ q,
                                   const int* __restrict__ id, const int* __restrict__ sp,
                                   GridDev g, double4* __restrict__ sxyzq,
                                   int* __restrict__ sid, int* __restrict__ ssp,
                                   int* __restrict__ perm, const double* __restrict__ w3,
                                   int64_t w3_stride, double* __restrict__ sw3,
                                   int64_t sw3_stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int d = start[ion_bin[i]] + ion_rank[i];
    if (d < 0 || d >= n) return;  // ranks are a permutation of each bin's slots
    double xi = x[i], yi = y[i];
    if (isfinite(xi) && isfinite(yi)) {
        xi = reduce_periodic(xi, g.Lx);
        yi = reduce_periodic(yi, g.Ly);
    }
    sxyzq[d] = make_double4(xi, yi, z[i], q ? q[i] : 0.0);
    if (id) sid[d] = id[i];
    if (sp) ssp[d] = sp[i];
    if (w3) {
        sw3[d] = w3[i];
        sw3[d + sw3_stride] = w3[i + w3_stride];
        sw3[d + 2 * sw3_stride] = w3[i + 2 * w3_stride];
    }
    perm[d] = i;
}

int build_cell_list(Ctx* c, int n, const double* x, const double* y, const double* z,
                    const double* q, const int* id, const int* sp, hipStream_t s,
                    const double* w3, int64_t w3_stride) {
    ++c->cl_gen;
    const GridDev& g = c->gd;
    const int64_t nb = c->nbins;
    const int T = 256;
    if (n > 0)
        bin_count_kernel<<<(n + T - 1) / T, T, 0, s>>>(g, n, x, y, z, c->bin_count, c->ion_bin,
                                                       c->ion_rank, c->flags);
    scan_counts(c->bin_count, nb, c->scan_tmp, c->bin_start, s);
    if (n > 0)
        bin_scatter_kernel<<<(n + T - 1) / T, T, 0, s>>>(n, c->ion_bin, c->ion_rank, c->bin_start,
                                                         x, y, z, q, id, sp, g, c->sxyzq,
                                                         c->sid, c->ssp, c->perm, w3, w3_stride,
                                                         c->fp, c->n_max);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int batch_cell_list(Batch* b, const double* pos, const double* q, const int* id, const int* sp,
                    hipStream_t s) {
    const int64_t nb = b->nbins_tot;
    const int n = (int)b->n_tot;
    const int T = b->cfg.ion_block;
    bin_count_batch_kernel<<<(n + T - 1) / T, T, 0, s>>>(b->reps_d, b->ion_rep, n, pos, pos + n,
                                                         pos + 2 * (int64_t)n, b->bin_count,
                                                         b->ion_bin, b->ion_rank, b->flags);
    scan_counts(b->bin_count, nb, b->scan_tmp, b->bin_start, s);
    bin_scatter_batch_kernel<<<(n + T - 1) / T, T, 0, s>>>(b->reps_d, b->ion_rep, n, b->ion_bin,
                                                           b->ion_rank, b->bin_start, pos, pos + n,
                                                           pos + 2 * (int64_t)n, q, id, sp, b->sxyzq,
                                                           b->sid, b->ssp, b->perm);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

void fill_f64(double* a, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    fill_f64_kernel<<<(int)std::min<int64_t>((n + 255) / 256, 8192), 256, 0, s>>>(a, n, v);
}

}  // namespace discos
