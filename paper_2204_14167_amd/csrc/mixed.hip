// The Poisson solve with walls of mixed type (Sec. IV.B: a metal strip on a dielectric
// wall; Sec. II.B.1: the wall data may vary along the wall).
//
// A wall whose columns differ in type has a ghost rule that varies with (x, y): the
// layer next to it no longer has the same diagonal in every column, and the in-plane
// Fourier modes couple.  A = -eps lap_h with each column's homogeneous ghost differs from
// M, the same operator with a uniform wall pair (per wall Dirichlet if the wall has any
// Dirichlet column, else Neumann; positive definite), only on the diagonal of the wall
// layer cells of the other columns: A = M + U C U^T with U selecting those cells and
// C = -2 eps / h^2 on each (a Neumann ghost +phi_0 where M has -phi_0).  By the
// Sherman-Morrison-Woodbury identity
//   A^-1 b = u - M^-1 U y,   u = M^-1 b,   (C^-1 + U^T M^-1 U) y = U^T u,
// so the solve takes two uniform-wall solves (the per-mode FFT / tridiagonal solve) and
// a system on the wall layers only.  There, M^-1 restricted to the two wall layers is a
// 2 x 2 map per in-plane Fourier mode (the wall rows and columns of the inverse of the
// mode's tridiagonal matrix), so the capacitance operator S = C^-1 + U^T M^-1 U costs two
// 2-D FFTs of the wall planes.  -S is symmetric positive definite (A^-1 >= M^-1) and is
// solved by conjugate gradients, preconditioned with the same per-mode inverse as if the
// whole wall were of the other type ((1 / 2c) I - G_k inverted per mode; the mode where
// that is singular, both walls Neumann at kappa = 0, is shifted).  Ten to twenty-five
// iterations reach the tolerance on the strips and random maps of the tests.
//
// Reductions use a fixed grid and a fixed order (deterministic), and the scalars of the
// iteration stay on the device; the host reads the residual every few iterations.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace discos {

#define MX_THREADS 256
#define MX_CHECK 4          // iterations between convergence tests on the host
#define MX_MAX_ITER 500
#define MX_TOL 1e-14        // relative residual of the capacitance system

enum { S_BB = 0, S_RR, S_PQ, S_RZ, S_RZN, S_NUM };

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[MX_THREADS];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = MX_THREADS / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    return red[0];
}

// ---- the per-mode tables --------------------------------------------------------------
// (T^-1)_00, (T^-1)_0L, (T^-1)_LL of the mode's tridiagonal matrix T (diagonal 2 + lam,
// off-diagonals -1, the wall rows' diagonals less the ghost signs s_lo, s_hi): the first
// by the continued fraction of the pivots from the top down, the others from the
// bottom up (T^-1_0L is the product of the inverse pivots times T^-1_LL).
__device__ void wall_green(int nz, double lam, double s_lo, double s_hi, double& g00, double& g0l,
                           double& gll) {
    const double d = 2.0 + lam;
    double a = d - s_hi;  // pivots from the top layer down
    for (int k = nz - 2; k >= 1; --k) a = d - 1.0 / a;
    g00 = 1.0 / (d - s_lo - 1.0 / a);
    double t = d - s_lo;  // pivots from the bottom layer up
    double prod = 1.0 / t;
    for (int k = 1; k < nz - 1; ++k) {
        t = d - 1.0 / t;
        prod /= t;
    }
    t = d - s_hi - 1.0 / t;
    gll = 1.0 / t;
    g0l = prod * gll;
}

__device__ __forceinline__ double mode_lambda(int m, int j, int nx, int ny) {
    return (2.0 - 2.0 * cos(2.0 * M_PI * m / nx)) + (2.0 - 2.0 * cos(2.0 * M_PI * j / ny));
}

// G = M^-1 on the wall layers and P = ((1 / 2c) I - G)^-1 per mode (t = j (nx/2+1) + m),
// the rows of walls without unknowns replaced by the identity.
__global__ void cap_table_kernel(GridDev g, double inv_c, double s_lo, double s_hi, int use_lo,
                                 int use_hi, double* __restrict__ G, double* __restrict__ P) {
    const int nmode = g.nxh * g.ny;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nmode) return;
    const int m = t % g.nxh, j = t / g.nxh;
    double g00, g0l, gll;
    wall_green(g.nz, mode_lambda(m, j, g.nx, g.ny), s_lo, s_hi, g00, g0l, gll);
    g00 *= inv_c;
    g0l *= inv_c;
    gll *= inv_c;
    G[t] = g00;
    G[nmode + t] = g0l;
    G[2 * nmode + t] = gll;
    const double hc = 0.5 * inv_c;
    auto q_of = [&](double a00, double a0l, double all, double& q00, double& q01, double& q11) {
        q00 = use_lo ? hc - a00 : 1.0;
        q11 = use_hi ? hc - all : 1.0;
        q01 = (use_lo && use_hi) ? -a0l : 0.0;
    };
    double q00, q01, q11;
    q_of(g00, g0l, gll, q00, q01, q11);
    double det = q00 * q11 - q01 * q01;
    if (!(det > 1e-12 * (fabs(q00 * q11) + q01 * q01))) {
        // singular (kappa = 0 between Neumann walls): shifted by a third of the
        // neighbouring mode's diagonal
        double h00, h0l, hll, r00, r01, r11;
        wall_green(g.nz, mode_lambda(g.nxh > 1 ? 1 : 0, g.nxh > 1 ? 0 : 1, g.nx, g.ny), s_lo, s_hi, h00,
                   h0l, hll);
        q_of(h00 * inv_c, h0l * inv_c, hll * inv_c, r00, r01, r11);
        const double eps = 0.3 * fmin(use_lo ? r00 : r11, use_hi ? r11 : r00);
        if (use_lo) q00 += eps;
        if (use_hi) q11 += eps;
        det = q00 * q11 - q01 * q01;
    }
    P[t] = q11 / det;
    P[nmode + t] = -q01 / det;
    P[2 * nmode + t] = q00 / det;
}

// ---- vectors on the two wall planes ([2][ny][nx]) ----------------------------------------
// A wall-plane cell is an unknown when its column's type differs from the wall's
// reference type.
__device__ __forceinline__ bool cap_unknown(const WallDev& w, const int ref[2], int64_t e, int64_t ncol) {
    const int wall = e >= ncol ? 1 : 0;
    const int64_t col = e - wall * ncol;
    return w.map[wall] != nullptr && w.map[wall][col] != ref[wall];
}

struct CapRef {
    int r[2];
};

// r = -U^T u (the wall layers of u at the unknowns), y = 0; part = sums of r r.
__global__ void __launch_bounds__(MX_THREADS)
cap_rhs_kernel(GridDev g, WallDev w, CapRef ref, const double* __restrict__ u, double* __restrict__ r,
               double* __restrict__ y, double* __restrict__ part) {
    const int64_t ncol = (int64_t)g.nx * g.ny, n2 = 2 * ncol;
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)MX_THREADS + threadIdx.x; e < n2;
         e += (int64_t)gridDim.x * MX_THREADS) {
        const int wall = e >= ncol ? 1 : 0;
        const int64_t col = e - wall * ncol;
        const double v = cap_unknown(w, ref.r, e, ncol)
                             ? -u[(wall ? (int64_t)(g.nz - 1) * ncol : 0) + col]
                             : 0.0;
        r[e] = v;
        y[e] = 0.0;
        acc += v * v;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// q = -S p = (1 / 2c) p - U^T K p at the unknowns (kp: M^-1 p on the wall planes, before
// the restriction); part = sums of p q.
__global__ void __launch_bounds__(MX_THREADS)
cap_combine_kernel(GridDev g, WallDev w, CapRef ref, double hc, const double* __restrict__ p,
                   const double* __restrict__ kp, double* __restrict__ q, double* __restrict__ part) {
    const int64_t ncol = (int64_t)g.nx * g.ny, n2 = 2 * ncol;
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)MX_THREADS + threadIdx.x; e < n2;
         e += (int64_t)gridDim.x * MX_THREADS) {
        const double v = cap_unknown(w, ref.r, e, ncol) ? hc * p[e] - kp[e] : 0.0;
        q[e] = v;
        acc += p[e] * v;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// z = the unknowns of pz (the preconditioned residual); part = sums of r z.
__global__ void __launch_bounds__(MX_THREADS)
cap_restrict_dot_kernel(GridDev g, WallDev w, CapRef ref, const double* __restrict__ pz,
                        const double* __restrict__ r, double* __restrict__ z, double* __restrict__ part) {
    const int64_t ncol = (int64_t)g.nx * g.ny, n2 = 2 * ncol;
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)MX_THREADS + threadIdx.x; e < n2;
         e += (int64_t)gridDim.x * MX_THREADS) {
        const double v = cap_unknown(w, ref.r, e, ncol) ? pz[e] : 0.0;
        z[e] = v;
        acc += r[e] * v;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// S[slot] = sum of the partials (fixed order); with roll, also S[RZ] = S[RZN] first.
__global__ void __launch_bounds__(MX_THREADS)
mx_finish_kernel(const double* __restrict__ part, int nparts, double* __restrict__ S, int slot,
                 int roll) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < nparts; k += MX_THREADS) acc += part[k];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) {
        if (roll) S[S_RZ] = S[S_RZN];
        S[slot] = t;
    }
}

// alpha = S[RZ] / S[PQ]; x += alpha p; r -= alpha q; part = sums of r r.
__global__ void __launch_bounds__(MX_THREADS)
mx_step_kernel(int64_t n, const double* __restrict__ S, const double* __restrict__ p,
               const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r,
               double* __restrict__ part) {
    const double alpha = S[S_PQ] != 0.0 ? S[S_RZ] / S[S_PQ] : 0.0;
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)MX_THREADS + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * MX_THREADS) {
        x[e] += alpha * p[e];
        const double v = r[e] - alpha * q[e];
        r[e] = v;
        acc += v * v;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// p = z + beta p, beta = S[RZN] / S[RZ] (first: p = z).
__global__ void __launch_bounds__(MX_THREADS)
mx_direction_kernel(int64_t n, const double* __restrict__ S, int first,
                    const double* __restrict__ z, double* __restrict__ p) {
    const double beta = (first || S[S_RZ] == 0.0) ? 0.0 : S[S_RZN] / S[S_RZ];
    for (int64_t e = blockIdx.x * (int64_t)MX_THREADS + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * MX_THREADS)
        p[e] = z[e] + (first ? 0.0 : beta * p[e]);
}

// f = U y on the wall layers of a zero volume (the right-hand side of the second
// uniform-wall solve).
__global__ void cap_place_kernel(GridDev g, const double* __restrict__ y, double* __restrict__ f) {
    const int64_t ncol = (int64_t)g.nx * g.ny, n = ncol * g.nz;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / ncol, col = e - k * ncol;
        double v = 0.0;
        if (k == 0) v += y[col];
        if (k == g.nz - 1) v += y[ncol + col];
        f[e] = v;
    }
}

// phi -= v.
__global__ void cap_sub_kernel(int64_t n, const double* __restrict__ v, double* __restrict__ phi) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        phi[e] -= v[e];
}

// ---- the direct solve --------------------------------------------------------------
// The capacitance system lives on the wall cells only, and its operator
// -S = (1 / 2c) I - U^T M^-1 U is fixed by the maps, the wall types and eps.  Its entries
// follow from the wall Green's functions: (U^T M^-1 U)_ij = g_ab(x_i - x_j) for unknown i
// on wall plane b and unknown j on wall plane a, with g_ab(d) the response on plane b to
// a unit source at the origin of plane a (the uniform-wall operator is invariant under
// in-plane periodic shifts), read off two filter passes of unit sources.  -S is factorised
// once per set of maps (Cholesky) and inverted; a solve is then one product with the
// inverse, about 8 n^2 bytes read, in place of 10 to 25 preconditioned iterations of two
// filter passes each.

// out = the unit vector at e (n entries).
__global__ void cap_unit_kernel(int64_t n, int64_t e, double* __restrict__ out) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        out[k] = k == e ? 1.0 : 0.0;
}

// A[i + j nd] = (1 / 2c) [i = j] - g_{a b}(x_i - x_j), a the plane of unknown j, b that of
// unknown i (t0, t1: the responses [2][ny][nx] to unit sources at the origin of plane 0, 1).
__global__ void cap_dense_assemble_kernel(GridDev g, int nd, const int* __restrict__ idx,
                                          const double* __restrict__ t0,
                                          const double* __restrict__ t1, double hc,
                                          double* __restrict__ A) {
    const int64_t ncol = (int64_t)g.nx * g.ny, total = (int64_t)nd * nd;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / nd), i = (int)(e - (int64_t)j * nd);
        const int ei = idx[i], ej = idx[j];
        const int bi = ei >= ncol ? 1 : 0, aj = ej >= ncol ? 1 : 0;
        const int ci = ei - bi * (int)ncol, cj = ej - aj * (int)ncol;
        const int dx = ((ci % g.nx) - (cj % g.nx)) & (g.nx - 1);
        const int dy = ((ci / g.nx) - (cj / g.nx)) & (g.ny - 1);
        const double* t = aj ? t1 : t0;
        A[e] = (i == j ? hc : 0.0) - t[bi * ncol + (int64_t)dy * g.nx + dx];
    }
}

// The upper triangle from the lower one.
__global__ void cap_symmetrize_kernel(int nd, double* __restrict__ A) {
    const int64_t total = (int64_t)nd * nd;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / nd), i = (int)(e - (int64_t)j * nd);
        if (i < j) A[e] = A[j + (int64_t)i * nd];
    }
}

// rv = -U^T u on the unknowns (u's wall layers).
__global__ void cap_dense_pack_kernel(GridDev g, int nd, const int* __restrict__ idx,
                                      const double* __restrict__ u, double* __restrict__ rv) {
    const int64_t ncol = (int64_t)g.nx * g.ny;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x) {
        const int e = idx[i];
        const int wall = e >= ncol ? 1 : 0;
        rv[i] = -u[(wall ? (int64_t)(g.nz - 1) * ncol : 0) + (e - wall * ncol)];
    }
}

// yv = A rv with A symmetric: output i is column i's product with rv, one wavefront per
// output (its lanes along the column, coalesced), summed in a fixed order.
__global__ void __launch_bounds__(256) cap_dense_gemv_kernel(int nd, const double* __restrict__ A,
                                                             const double* __restrict__ rv,
                                                             double* __restrict__ yv) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nd) return;
    const double* col = A + (size_t)i * nd;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = lane;
    for (; j + 192 < nd; j += 256) {
        a0 += col[j] * rv[j];
        a1 += col[j + 64] * rv[j + 64];
        a2 += col[j + 128] * rv[j + 128];
        a3 += col[j + 192] * rv[j + 192];
    }
    for (; j < nd; j += 64) a0 += col[j] * rv[j];
    double acc = (a0 + a1) + (a2 + a3);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) yv[i] = acc;
}

// y[idx[i]] = yv[i] (y cleared before).
__global__ void cap_dense_scatter_kernel(int nd, const int* __restrict__ idx,
                                         const double* __restrict__ yv, double* __restrict__ y) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x)
        y[idx[i]] = yv[i];
}

bool release_dense_capacitance(Ctx* c) {
    bool ok = true;
    if (c->cap_inv) ok = hipFree(c->cap_inv) == hipSuccess && ok;
    if (c->cap_idx) ok = hipFree(c->cap_idx) == hipSuccess && ok;
    if (c->cap_vec) ok = hipFree(c->cap_vec) == hipSuccess && ok;
    c->cap_inv = nullptr;
    c->cap_idx = nullptr;
    c->cap_vec = nullptr;
    c->cap_alloc = 0;
    c->cap_nd = -1;
    if (c->rb) {
        ok = rocblas_destroy_handle(static_cast<rocblas_handle>(c->rb)) == rocblas_status_success && ok;
        c->rb = nullptr;
    }
    return ok;
}

// The inverse of -S for the present maps (cap_nd unknowns), formed when the maps, wall
// types or eps changed and there are at most DISCOS_MIXED_DENSE_MAX unknowns.  cap_nd = 0
// (the iterative solve) otherwise, with DISCOS_CREATE_MIXED_ITERATIVE, or when memory
// or the factorisation fails.  tmp: 3 wall-plane pairs of scratch.
static int prepare_dense(Ctx* c, const int ref[2], int key, double eps, double hc,
                         const double* G, double* tmp, hipStream_t s) {
    if (c->cap_nd >= 0 && c->cap_dkey == key && c->cap_dgen == c->wm_gen && c->cap_deps == eps)
        return DISCOS_OK;
    c->cap_nd = 0;
    c->cap_dkey = key;
    c->cap_dgen = c->wm_gen;
    c->cap_deps = eps;
    if (c->mx_iterative) return DISCOS_OK;
    const GridDev& g = c->gd;
    const int64_t ncol = (int64_t)g.nx * g.ny, n2 = 2 * ncol;
    std::vector<int> idx;
    for (int w = 0; w < 2; ++w) {
        const std::vector<int32_t>& m = c->wm_host[w];
        if ((int64_t)m.size() != ncol) continue;
        for (int64_t col = 0; col < ncol; ++col)
            if (m[col] != ref[w]) idx.push_back((int)(w * ncol + col));
    }
    const int nd = (int)idx.size();
    if (nd == 0 || nd > DISCOS_MIXED_DENSE_MAX) return DISCOS_OK;
    if (hipStreamSynchronize(s) != hipSuccess) return DISCOS_E_HIP;
    if (nd > c->cap_alloc) {
        rocblas_handle keep = static_cast<rocblas_handle>(c->rb);
        c->rb = nullptr;
        if (!release_dense_capacitance(c)) return DISCOS_E_HIP;
        c->rb = keep;
        c->cap_nd = 0;
        if (hipMalloc(&c->cap_inv, (size_t)nd * nd * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->cap_idx, (size_t)(nd + 1) * sizeof(int)) != hipSuccess ||
            hipMalloc(&c->cap_vec, (size_t)2 * nd * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();  // out of memory: the iterative solve needs none of it
            keep = static_cast<rocblas_handle>(c->rb);
            c->rb = nullptr;
            release_dense_capacitance(c);
            c->rb = keep;
            c->cap_nd = 0;
            return DISCOS_OK;
        }
        c->cap_alloc = nd;
    }
    if (!c->rb) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return DISCOS_OK;
        c->rb = h;
    }
    rocblas_handle h = static_cast<rocblas_handle>(c->rb);
    if (hipMemcpy(c->cap_idx, idx.data(), (size_t)nd * sizeof(int), hipMemcpyHostToDevice) !=
        hipSuccess)
        return DISCOS_E_HIP;
    // the Green's functions: responses to unit sources at the origins of the two planes
    double* src = tmp;
    double* t0 = tmp + n2;
    double* t1 = tmp + 2 * n2;
    const int nbu = (int)std::min<int64_t>((n2 + 255) / 256, 4096);
    cap_unit_kernel<<<nbu, 256, 0, s>>>(n2, 0, src);
    int rc = plane_pair_filter(c, src, t0, G, s);
    if (rc) return rc;
    cap_unit_kernel<<<nbu, 256, 0, s>>>(n2, ncol, src);
    rc = plane_pair_filter(c, src, t1, G, s);
    if (rc) return rc;
    const int64_t total = (int64_t)nd * nd;
    const int nba = (int)std::min<int64_t>((total + 255) / 256, 65536);
    cap_dense_assemble_kernel<<<nba, 256, 0, s>>>(g, nd, c->cap_idx, t0, t1, hc, c->cap_inv);
    if (hipGetLastError() != hipSuccess) return DISCOS_E_HIP;
    // -S = L L^T, then its inverse from the factor (lower triangle), then the upper half
    rocblas_int* info = reinterpret_cast<rocblas_int*>(c->cap_idx + nd);
    if (rocblas_set_stream(h, s) != rocblas_status_success ||
        rocsolver_dpotrf(h, rocblas_fill_lower, nd, c->cap_inv, nd, info) != rocblas_status_success)
        return DISCOS_E_HIP;
    rocblas_int ih = 0;
    if (hipMemcpyAsync(&ih, info, sizeof(ih), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return DISCOS_E_HIP;
    if (ih != 0) return DISCOS_OK;  // not positive definite in floating point: iterate
    if (rocsolver_dpotri(h, rocblas_fill_lower, nd, c->cap_inv, nd, info) != rocblas_status_success)
        return DISCOS_E_HIP;
    if (hipMemcpyAsync(&ih, info, sizeof(ih), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return DISCOS_E_HIP;
    if (ih != 0) return DISCOS_OK;
    cap_symmetrize_kernel<<<nba, 256, 0, s>>>(nd, c->cap_inv);
    if (hipGetLastError() != hipSuccess) return DISCOS_E_HIP;
    c->cap_nd = nd;
    return DISCOS_OK;
}

// The capacitance system by preconditioned conjugate gradients: r = -U^T u, y = 0, then
// iterate to the tolerance.
static int solve_capacitance_cg(Ctx* c, const GridDev& g, const WallDev& w, const CapRef& cr,
                                const double* G, const double* P, int nb, double* S,
                                double* part, const double* phi, double* y, double* r, double* pd,
                                double* z, double* q, double* t, hipStream_t s) {
    const int64_t n2 = 2 * (int64_t)g.nx * g.ny;
    const double cst = c->cap_eps / (c->grid.h * c->grid.h);
    auto finish = [&](int slot, int roll) {
        mx_finish_kernel<<<1, MX_THREADS, 0, s>>>(part, nb, S, slot, roll);
    };
    int rc = DISCOS_OK;
    cap_rhs_kernel<<<nb, MX_THREADS, 0, s>>>(g, w, cr, phi, r, y, part);
    finish(S_BB, 0);
    // z = P r (restricted), p = z
    rc = plane_pair_filter(c, r, t, P, s);
    if (rc) return rc;
    cap_restrict_dot_kernel<<<nb, MX_THREADS, 0, s>>>(g, w, cr, t, r, z, part);
    finish(S_RZN, 0);
    mx_direction_kernel<<<nb, MX_THREADS, 0, s>>>(n2, S, 1, z, pd);
    // the host reads the residual every MX_CHECK iterations, from a few iterations short
    // of the last solve's count on (each read waits for the stream)
    const int first_check = std::max(MX_CHECK, (c->mx_iters - 2 * MX_CHECK) / MX_CHECK * MX_CHECK);
    bool done = false;
    for (int it = 1; it <= MX_MAX_ITER && !done; ++it) {
        rc = plane_pair_filter(c, pd, t, G, s);  // M^-1 p on the wall planes
        if (rc) return rc;
        cap_combine_kernel<<<nb, MX_THREADS, 0, s>>>(g, w, cr, 0.5 / cst, pd, t, q, part);
        finish(S_PQ, 1);
        mx_step_kernel<<<nb, MX_THREADS, 0, s>>>(n2, S, pd, q, y, r, part);
        finish(S_RR, 0);
        if (hipGetLastError() != hipSuccess) return DISCOS_E_HIP;
        if ((it >= first_check && it % MX_CHECK == 0) || it == MX_MAX_ITER) {
            double h[2];
            if (hipMemcpyAsync(h, S, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return DISCOS_E_HIP;
            if (!(std::isfinite(h[S_RR]) && std::isfinite(h[S_BB]))) return DISCOS_E_NONFINITE;
            if (h[S_RR] <= MX_TOL * MX_TOL * h[S_BB]) {
                c->mx_iters = it;
                done = true;
                break;
            }
            if (it == MX_MAX_ITER) return DISCOS_E_NOT_CONVERGED;
        }
        rc = plane_pair_filter(c, r, t, P, s);
        if (rc) return rc;
        cap_restrict_dot_kernel<<<nb, MX_THREADS, 0, s>>>(g, w, cr, t, r, z, part);
        finish(S_RZN, 0);
        mx_direction_kernel<<<nb, MX_THREADS, 0, s>>>(n2, S, 0, z, pd);
    }
    if (!done) return DISCOS_E_NOT_CONVERGED;
    return DISCOS_OK;
}

int solve_poisson_mixed(Ctx* c, const double* rhs, const discos_params* p, const int ref[2],
                        double* phi, hipStream_t s) {
    const GridDev& g = c->gd;
    const WallDev w = wall_of(p);
    const int64_t n = c->ncell, ncol = (int64_t)g.nx * g.ny, n2 = 2 * ncol;
    const int nmode = g.nxh * g.ny;
    const double cst = p->eps / (c->grid.h * c->grid.h);
    const int nb = (int)std::min<int64_t>((n2 + MX_THREADS - 1) / MX_THREADS, PART_MAX);
    const int nbv = (int)std::min<int64_t>((n + 255) / 256, 4096);
    double* G = c->cap;
    double* P = c->cap + 3 * (size_t)nmode;
    double* y = c->cap + 6 * (size_t)nmode;
    double* r = y + n2;
    double* pd = r + n2;
    double* z = pd + n2;
    double* q = z + n2;
    double* t = q + n2;
    double* S = c->pcg_s;
    double* part = c->part;
    const CapRef cr{{ref[0], ref[1]}};
    // the uniform pair of reference types, no maps
    discos_params pu = *p;
    pu.bc_type[0] = ref[0];
    pu.bc_type[1] = ref[1];
    pu.bc_type_map[0] = pu.bc_type_map[1] = nullptr;
    const int use_lo = p->bc_type_map[0] != nullptr, use_hi = p->bc_type_map[1] != nullptr;
    const int key = ref[0] + 2 * ref[1] + 4 * use_lo + 8 * use_hi;
    if (c->cap_key != key || c->cap_eps != p->eps) {
        cap_table_kernel<<<(nmode + 255) / 256, 256, 0, s>>>(
            g, 1.0 / cst, ref[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0,
            ref[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0, use_lo, use_hi, G, P);
        c->cap_key = key;
        c->cap_eps = p->eps;
    }
    int rc = prepare_dense(c, ref, key, p->eps, 0.5 / cst, G, r, s);
    if (rc) return rc;
    // u = M^-1 b into phi (b may share storage with phi)
    rc = solve_poisson(c, rhs, &pu, phi, s);
    if (rc) return rc;
    if (c->cap_nd > 0) {
        // y = (-S)^-1 (-U^T u) by the held inverse
        const int nd = c->cap_nd;
        double* rv = c->cap_vec;
        double* yv = rv + nd;
        const int nbd = (nd + 255) / 256;
        cap_dense_pack_kernel<<<nbd, 256, 0, s>>>(g, nd, c->cap_idx, phi, rv);
        cap_dense_gemv_kernel<<<(nd + 3) / 4, 256, 0, s>>>(nd, c->cap_inv, rv, yv);
        fill_f64(y, n2, 0.0, s);
        cap_dense_scatter_kernel<<<nbd, 256, 0, s>>>(nd, c->cap_idx, yv, y);
    } else {
        rc = solve_capacitance_cg(c, g, w, cr, G, P, nb, S, part, phi, y, r, pd, z, q, t, s);
        if (rc) return rc;
    }
    // phi = u - M^-1 U y
    double* f = c->pcg;
    double* v = c->pcg + n;
    cap_place_kernel<<<nbv, 256, 0, s>>>(g, y, f);
    rc = solve_poisson(c, f, &pu, v, s);
    if (rc) return rc;
    cap_sub_kernel<<<nbv, 256, 0, s>>>(n, v, phi);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
