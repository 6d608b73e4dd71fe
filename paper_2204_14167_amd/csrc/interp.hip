// J^es: interpolation of the electric field E = -grad_h phi to the ions (eq efieldop,
// eq kernel1) with ghost values beyond the walls filled from the wall conditions
// (Sec. II.B.1: ghosts satisfy the boundary condition on phi).
//
// E lives on the faces of the cell-centred phi (the staggered location of grad_h);
// each component is gathered from its own face nodes, computing the face
// differences on the fly from phi, so E is never stored.
#include "kernels.h"

namespace discos {

// phi at cell (i, j, k), i and j already periodic, k in [-3, nz + 2]: ghost layer
// -1-m is 2 phi_b - phi_m (Dirichlet) or phi_m + (2m+1) h sigma / eps (Neumann);
// mirror rule at the top wall.
__device__ __forceinline__ double phi_at(const double* __restrict__ phi, const GridDev& g,
                                         const WallDev& w, int i, int j, int k) {
    if (k >= 0 && k < g.nz) return phi[((size_t)k * g.ny + j) * g.nx + i];
    const int wall = k < 0 ? 0 : 1;
    const int m = k < 0 ? -1 - k : k - g.nz;
    const int src = min(max(k < 0 ? m : g.nz - 1 - m, 0), g.nz - 1);
    const double base = phi[((size_t)src * g.ny + j) * g.nx + i];
    const double v = w.value[wall] ? w.value[wall][(size_t)j * g.nx + i] : 0.0;
    if (w.type[wall] == DISCOS_BC_DIRICHLET) return 2.0 * v - base;
    return base + (2 * m + 1) * g.h * v / w.eps;
}

__global__ void interp_es_kernel(GridDev g, WallDev w, int n, int op,
                                 const double* __restrict__ px, const double* __restrict__ py,
                                 const double* __restrict__ pz, const double* __restrict__ phi,
                                 const double* __restrict__ q, double ex0, double ex1, double ex2,
                                 double* __restrict__ out, int64_t out_stride,
                                 int* __restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = px[i], y = py[i], z = pz[i];
    if (!pos_ok(g, x, y, z)) {
        set_flag(flags, (isfinite(x) && isfinite(y) && isfinite(z)) ? DISCOS_FLAG_OUT_OF_DOMAIN
                                                                  : DISCOS_FLAG_NONFINITE);
        if (op == DISCOS_INTERP_PHI) {
            out[i] = 0.0;
        } else {
            out[i] = 0.0;
            out[i + out_stride] = 0.0;
            out[i + 2 * out_stride] = 0.0;
        }
        return;
    }
    const double xr = reduce_periodic(x, g.Lx) * g.inv_h;
    const double yr = reduce_periodic(y, g.Ly) * g.inv_h;
    const double zr = z * g.inv_h;
    int icx, icy, icz;
    double wcx[4], wcy[4], wcz[4];
    peskin4(xr - 0.5, icx, wcx);
    peskin4(yr - 0.5, icy, wcy);
    peskin4(zr - 0.5, icz, wcz);
    int jx[4], jy[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) jx[a] = wrapi(icx + a, g.nx);
#pragma unroll
    for (int b = 0; b < 4; ++b) jy[b] = wrapi(icy + b, g.ny);

    if (op == DISCOS_INTERP_PHI) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double row = 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a) row += wcx[a] * phi_at(phi, g, w, jx[a], jy[b], icz + c);
                acc += wcz[c] * wcy[b] * row;
            }
        out[i] = acc;
        return;
    }

    int ifx, ify, ifz;
    double wfx[4], wfy[4], wfz[4];
    peskin4(xr, ifx, wfx);
    peskin4(yr, ify, wfy);
    peskin4(zr, ifz, wfz);
    const double mih = -g.inv_h;

    // E_x on x-faces (i h, (j+1/2) h, (k+1/2) h): face a uses cells a-1 and a
    double Ex = 0.0;
    {
        int cx[5];
#pragma unroll
        for (int a = 0; a < 5; ++a) cx[a] = wrapi(ifx - 1 + a, g.nx);
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double v[5];
#pragma unroll
                for (int a = 0; a < 5; ++a) v[a] = phi_at(phi, g, w, cx[a], jy[b], icz + c);
                double row = 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a) row += wfx[a] * (mih * (v[a + 1] - v[a]));
                Ex += wcz[c] * wcy[b] * row;
            }
    }
    // E_y on y-faces
    double Ey = 0.0;
    {
        int cy[5];
#pragma unroll
        for (int b = 0; b < 5; ++b) cy[b] = wrapi(ify - 1 + b, g.ny);
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double v[5];
#pragma unroll
                for (int b = 0; b < 5; ++b) v[b] = phi_at(phi, g, w, jx[a], cy[b], icz + c);
                double row = 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) row += wfy[b] * (mih * (v[b + 1] - v[b]));
                Ey += wcz[c] * wcx[a] * row;
            }
    }
    // E_z on z-faces ((i+1/2) h, (j+1/2) h, k h): face c uses cells c-1 and c (ghosts)
    double Ez = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double v[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) v[c] = phi_at(phi, g, w, jx[a], jy[b], ifz - 1 + c);
            double col = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) col += wfz[c] * (mih * (v[c + 1] - v[c]));
            Ez += wcy[b] * wcx[a] * col;
        }
    if (op == DISCOS_INTERP_FORCE) {
        const double qi = q[i];
        Ex = qi * (Ex + ex0);
        Ey = qi * (Ey + ex1);
        Ez = qi * (Ez + ex2);
    }
    out[i] = Ex;
    out[i + out_stride] = Ey;
    out[i + 2 * out_stride] = Ez;
}

int interp_es(Ctx* c, int op, int n, const double* x, const double* y, const double* z,
              const double* phi, const double* q, const discos_params* p, double* out,
              int64_t out_stride, hipStream_t s) {
    if (n <= 0) return DISCOS_OK;
    const int T = 256;
    interp_es_kernel<<<(n + T - 1) / T, T, 0, s>>>(c->gd, wall_of(p), n, op, x, y, z, phi, q,
                                                   p->e_ext[0], p->e_ext[1], p->e_ext[2], out,
                                                   out_stride, c->flags);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
