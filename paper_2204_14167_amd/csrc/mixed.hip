// The Poisson solve with walls of mixed type (Sec. IV.B: a metal strip on a dielectric
// wall; Sec. II.B.1: the wall data may vary along the wall).
//
// A wall whose columns differ in type has a ghost rule that varies with (x, y): the
// layer next to it no longer has the same diagonal in every column, and the in-plane
// Fourier modes couple.  The system A phi = rhs (A = -eps lap_h with each column's
// homogeneous ghost; symmetric, and positive definite because such a wall has a
// Dirichlet column) is solved by conjugate gradients preconditioned with the per-mode
// FFT / tridiagonal solve of a uniform wall pair: per wall, Dirichlet if the wall has any
// Dirichlet column, else Neumann.  A differs from that operator only on the wall layers of
// the columns of the other type, so the preconditioned spectrum is one plus a
// perturbation living on those columns.
//
// Reductions use a fixed grid and a fixed order (deterministic), and the scalars of the
// iteration stay on the device; the host reads the residual every few iterations.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace discos {

#define MX_THREADS 256
#define MX_CHECK 4          // iterations between convergence tests on the host
#define MX_MAX_ITER 1000
#define MX_TOL 1e-13        // relative residual ||b - A x|| / ||b||

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

// (A v)(i, j, k) with the column's ghost sign below layer 0 and above layer nz - 1.
__device__ __forceinline__ double apply_at(const GridDev& g, const WallDev& w, double c,
                                           const double* __restrict__ v, int64_t e) {
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((int64_t)nx * ny));
    const int64_t plane = (int64_t)nx * ny;
    const double vc = v[e];
    double s = v[e - i + ((i + 1) & (nx - 1))] + v[e - i + ((i - 1) & (nx - 1))] +
               v[e - (int64_t)j * nx + (int64_t)((j + 1) & (ny - 1)) * nx] +
               v[e - (int64_t)j * nx + (int64_t)((j - 1) & (ny - 1)) * nx];
    s += k > 0 ? v[e - plane]
               : (wall_type_at(w, 0, i, j, nx) == DISCOS_BC_DIRICHLET ? -vc : vc);
    s += k < nz - 1 ? v[e + plane]
                    : (wall_type_at(w, 1, i, j, nx) == DISCOS_BC_DIRICHLET ? -vc : vc);
    return c * (6.0 * vc - s);
}

// q = A p; part[block] = sum p q over the block's cells.
__global__ void __launch_bounds__(MX_THREADS)
mx_apply_kernel(GridDev g, WallDev w, double c, int64_t n, const double* __restrict__ p,
                double* __restrict__ q, double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)MX_THREADS + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * MX_THREADS) {
        const double a = apply_at(g, w, c, p, e);
        q[e] = a;
        acc += p[e] * a;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// r = b - A x; part = sums of r r.
__global__ void __launch_bounds__(MX_THREADS)
mx_residual_kernel(GridDev g, WallDev w, double c, int64_t n, const double* __restrict__ x,
                   double* __restrict__ r, double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)MX_THREADS + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * MX_THREADS) {
        const double v = r[e] - apply_at(g, w, c, x, e);
        r[e] = v;
        acc += v * v;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// dst = src; part = sums of src src.
__global__ void __launch_bounds__(MX_THREADS)
mx_copy_kernel(int64_t n, const double* __restrict__ src, double* __restrict__ dst,
               double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)MX_THREADS + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * MX_THREADS) {
        const double v = src[e];
        dst[e] = v;
        acc += v * v;
    }
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// part = sums of a b.
__global__ void __launch_bounds__(MX_THREADS)
mx_dot_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
              double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)MX_THREADS + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * MX_THREADS)
        acc += a[e] * b[e];
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

int solve_poisson_mixed(Ctx* c, const double* rhs, const discos_params* p, const int ref[2],
                        double* phi, hipStream_t s) {
    const GridDev& g = c->gd;
    const WallDev w = wall_of(p);
    const int64_t n = c->ncell;
    const double cst = p->eps / (c->grid.h * c->grid.h);
    const int nb = (int)std::min<int64_t>((n + MX_THREADS - 1) / MX_THREADS, PART_MAX);
    double* r = c->pcg;
    double* pd = c->pcg + n;
    double* zq = c->pcg + 2 * n;
    double* S = c->pcg_s;
    double* part = c->part;
    // the preconditioner: the uniform pair of reference types, no maps
    discos_params pu = *p;
    pu.bc_type[0] = ref[0];
    pu.bc_type[1] = ref[1];
    pu.bc_type_map[0] = pu.bc_type_map[1] = nullptr;
    auto finish = [&](int slot, int roll) {
        mx_finish_kernel<<<1, MX_THREADS, 0, s>>>(part, nb, S, slot, roll);
    };
    // r = b (b may share storage with phi), x = M b, r = b - A x, z = M r, p = z.  In a
    // step, phi holds the previous step's potential (c->phi_warm): x starts from it, which
    // changes only the iteration count (the result is the solve to the same residual)
    const bool warm = phi == c->phi && rhs != phi && c->phi_warm;
    mx_copy_kernel<<<nb, MX_THREADS, 0, s>>>(n, rhs, r, part);
    finish(S_BB, 0);
    int rc = warm ? DISCOS_OK : solve_poisson(c, r, &pu, phi, s);
    if (rc) return rc;
    mx_residual_kernel<<<nb, MX_THREADS, 0, s>>>(g, w, cst, n, phi, r, part);
    finish(S_RR, 0);
    rc = solve_poisson(c, r, &pu, zq, s);
    if (rc) return rc;
    mx_dot_kernel<<<nb, MX_THREADS, 0, s>>>(n, r, zq, part);
    finish(S_RZN, 0);
    mx_direction_kernel<<<nb, MX_THREADS, 0, s>>>(n, S, 1, zq, pd);
    // the host reads the residual every MX_CHECK iterations, from a few iterations short
    // of the last solve's count on (each read waits for the stream)
    const int first_check = std::max(MX_CHECK, (c->mx_iters - 2 * MX_CHECK) / MX_CHECK * MX_CHECK);
    for (int it = 1; it <= MX_MAX_ITER; ++it) {
        mx_apply_kernel<<<nb, MX_THREADS, 0, s>>>(g, w, cst, n, pd, zq, part);
        finish(S_PQ, 1);
        mx_step_kernel<<<nb, MX_THREADS, 0, s>>>(n, S, pd, zq, phi, r, part);
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
                return DISCOS_OK;
            }
            if (it == MX_MAX_ITER) return DISCOS_E_NOT_CONVERGED;
        }
        rc = solve_poisson(c, r, &pu, zq, s);
        if (rc) return rc;
        mx_dot_kernel<<<nb, MX_THREADS, 0, s>>>(n, r, zq, part);
        finish(S_RZN, 0);
        mx_direction_kernel<<<nb, MX_THREADS, 0, s>>>(n, S, 0, zq, pd);
    }
    return DISCOS_E_NOT_CONVERGED;
}

}  // namespace discos
