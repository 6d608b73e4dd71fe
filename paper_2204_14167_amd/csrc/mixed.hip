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
    auto finish = [&](int slot, int roll) {
        mx_finish_kernel<<<1, MX_THREADS, 0, s>>>(part, nb, S, slot, roll);
    };
    // u = M^-1 b into phi (b may share storage with phi); r = -U^T u, y = 0
    int rc = solve_poisson(c, rhs, &pu, phi, s);
    if (rc) return rc;
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
