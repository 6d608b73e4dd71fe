// Poisson solve -eps lap_h phi = rhs with wall ghost rules (eq poisson, eqs esbc1-3).
//
// The 7-point operator is diagonal in the in-plane Fourier basis, leaving one
// tridiagonal system in z per mode (m, n) with
//   kappa^2 h^2 = 4 sin^2(pi m / nx) + 4 sin^2(pi n / ny).
// Passes: real FFT along x (two real rows packed into one complex FFT), complex FFT
// along y, Thomas solve along z (one thread per mode, coalesced across modes),
// inverse y, inverse real x.  All FFTs are radix-2 in LDS.  The paper solves the same
// discrete system with geometric multigrid; the direct solve gives it exactly.
#include "kernels.h"

namespace discos {

__device__ __forceinline__ int bitrev(int n, int logN) {
    return (int)(__brev((unsigned)n) >> (32 - logN));
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place radix-2 DIT FFTs of `lines` lines of length N stored back to back in LDS,
// input in bit-reversed order.  tw[k] = exp(-2 pi i k / N), k < N/2; `inv` conjugates.
__device__ void lds_fft(double2* a, int N, int logN, int lines, const double2* __restrict__ tw,
                        int inv) {
    const int halfN = N >> 1;
    const int nb = lines * halfN;
    for (int s = 1; s <= logN; ++s) {
        const int half = 1 << (s - 1);
        const int tstride = N >> s;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            const int line = b / halfN;
            const int bb = b - line * halfN;
            const int grp = bb / half;
            const int p = bb - grp * half;
            const int i = line * N + grp * 2 * half + p;
            const int j = i + half;
            double2 w = tw[p * tstride];
            if (inv) w.y = -w.y;
            const double2 u = a[i];
            const double2 v = cmul(a[j], w);
            a[i] = make_double2(u.x + v.x, u.y + v.y);
            a[j] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

#define FFT_THREADS 256

// Real rows (nrows of length nx, rows r and r+1 packed as one complex line) ->
// half spectra [nrows][nx/2 + 1].
__global__ void __launch_bounds__(FFT_THREADS)
fft_x_r2c_kernel(const double* __restrict__ in, double2* __restrict__ spec, int nx, int logN,
                 int npairs, int ppb, const double2* __restrict__ tw) {
    extern __shared__ double2 lds[];
    const int nxh = nx / 2 + 1;
    const int p0 = blockIdx.x * ppb;
    for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
        const int p = e / nx, n = e - p * nx;
        const int pr = p0 + p;
        double2 v = make_double2(0.0, 0.0);
        if (pr < npairs) {
            const size_t r0 = 2 * (size_t)pr;
            v = make_double2(in[r0 * nx + n], in[(r0 + 1) * nx + n]);
        }
        lds[p * nx + bitrev(n, logN)] = v;
    }
    __syncthreads();
    lds_fft(lds, nx, logN, ppb, tw, 0);
    for (int e = threadIdx.x; e < ppb * nxh; e += blockDim.x) {
        const int p = e / nxh, m = e - p * nxh;
        const int pr = p0 + p;
        if (pr >= npairs) continue;
        const double2 Z = lds[p * nx + (m % nx)];
        const double2 Zr = lds[p * nx + ((nx - m) % nx)];
        // A = (Z + conj Zr) / 2, B = (Z - conj Zr) / (2i)
        const double2 A = make_double2(0.5 * (Z.x + Zr.x), 0.5 * (Z.y - Zr.y));
        const double2 B = make_double2(0.5 * (Z.y + Zr.y), -0.5 * (Z.x - Zr.x));
        const size_t r0 = 2 * (size_t)pr;
        spec[r0 * nxh + m] = A;
        spec[(r0 + 1) * nxh + m] = B;
    }
}

// Half spectra -> real rows (inverse, unnormalised).
__global__ void __launch_bounds__(FFT_THREADS)
fft_x_c2r_kernel(const double2* __restrict__ spec, double* __restrict__ out, int nx, int logN,
                 int npairs, int ppb, const double2* __restrict__ tw) {
    extern __shared__ double2 lds[];
    const int nxh = nx / 2 + 1;
    const int p0 = blockIdx.x * ppb;
    for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
        const int p = e / nx, n = e - p * nx;
        const int pr = p0 + p;
        double2 z = make_double2(0.0, 0.0);
        if (pr < npairs) {
            const size_t r0 = 2 * (size_t)pr;
            double2 A, B;
            if (n < nxh) {
                A = spec[r0 * nxh + n];
                B = spec[(r0 + 1) * nxh + n];
            } else {
                const int m = nx - n;
                A = spec[r0 * nxh + m];
                B = spec[(r0 + 1) * nxh + m];
                A.y = -A.y;
                B.y = -B.y;
            }
            z = make_double2(A.x - B.y, A.y + B.x);  // A + i B
        }
        lds[p * nx + bitrev(n, logN)] = z;
    }
    __syncthreads();
    lds_fft(lds, nx, logN, ppb, tw, 1);
    for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
        const int p = e / nx, n = e - p * nx;
        const int pr = p0 + p;
        if (pr >= npairs) continue;
        const size_t r0 = 2 * (size_t)pr;
        const double2 z = lds[p * nx + n];
        out[r0 * nx + n] = z.x;
        out[(r0 + 1) * nx + n] = z.y;
    }
}

// Complex FFT along y of spec[k][j][m] for a block of MC consecutive m at one k.
__global__ void __launch_bounds__(FFT_THREADS)
fft_y_kernel(double2* __restrict__ spec, int nxh, int ny, int logN, int mc,
             const double2* __restrict__ tw, int inv) {
    extern __shared__ double2 lds[];
    const int m0 = blockIdx.x * mc;
    const size_t kbase = (size_t)blockIdx.y * ny * nxh;
    for (int e = threadIdx.x; e < mc * ny; e += blockDim.x) {
        const int c = e % mc, j = e / mc;
        const int m = m0 + c;
        lds[c * ny + bitrev(j, logN)] =
            (m < nxh) ? spec[kbase + (size_t)j * nxh + m] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    lds_fft(lds, ny, logN, mc, tw, inv);
    for (int e = threadIdx.x; e < mc * ny; e += blockDim.x) {
        const int c = e % mc, j = e / mc;
        const int m = m0 + c;
        if (m < nxh) spec[kbase + (size_t)j * nxh + m] = lds[c * ny + j];
    }
}

// Tridiagonal solve along z for every in-plane mode (one thread per mode).
// Rows (scaled by h^2 / eps): -x_{k-1} + (2 + kappa^2 h^2) x_k - x_{k+1} = r_k, with
// the ghost rule folded into the end rows (diag - s_lo, diag - s_hi).
// Mode (m, j) of a grid with nx, ny, nz: col and cpc point at its level-0 entries,
// levels st apart.
__device__ __forceinline__ void zsolve_mode(double2* __restrict__ col, double* __restrict__ cpc,
                                            size_t st, int m, int j, int nx, int ny, int nz,
                                            double scale, double s_lo, double s_hi, int singular,
                                            int* __restrict__ flags) {
    if (singular && m == 0 && j == 0) {
        // kappa = 0 with both walls Neumann: compatibility (neutrality), mean removal
        // (the projection onto the range), phi_0 pinned to 0, rows 1 .. nz-1 solved,
        // then shifted to mean(phi) = 0: the pseudo-inverse.
        double2 sum = make_double2(0.0, 0.0);
        double asum = 0.0;
        for (int k = 0; k < nz; ++k) {
            const double2 r = col[k * st];
            sum.x += r.x;
            sum.y += r.y;
            asum += sqrt(r.x * r.x + r.y * r.y);
        }
        if (singular == 1 && sqrt(sum.x * sum.x + sum.y * sum.y) > 1e-10 * fmax(asum, 1e-300))
            set_flag(flags, DISCOS_FLAG_NOT_NEUTRAL);
        const double2 mean = make_double2(sum.x / nz, sum.y / nz);
        // forward sweep over unknowns 1 .. nz-1 (diag 2, last row 1)
        double c_prev = 0.0;
        double2 d_prev = make_double2(0.0, 0.0);
        for (int k = 1; k < nz; ++k) {
            const double2 r0 = col[k * st];
            const double2 r = make_double2((r0.x - mean.x) * scale, (r0.y - mean.y) * scale);
            const double diag = (k == nz - 1) ? 1.0 : 2.0;
            const double den = (k == 1) ? diag : diag + c_prev;
            const double c = -1.0 / den;
            const double2 d = (k == 1) ? make_double2(r.x / den, r.y / den)
                                       : make_double2((r.x + d_prev.x) / den, (r.y + d_prev.y) / den);
            cpc[k * st] = c;
            col[k * st] = d;
            c_prev = c;
            d_prev = d;
        }
        double2 x = col[(nz - 1) * st];
        double2 xs = x;
        for (int k = nz - 2; k >= 1; --k) {
            const double2 d = col[k * st];
            const double c = cpc[k * st];
            x = make_double2(d.x - c * x.x, d.y - c * x.y);
            col[k * st] = x;
            xs.x += x.x;
            xs.y += x.y;
        }
        col[0] = make_double2(0.0, 0.0);
        const double2 shift = make_double2(xs.x / nz, xs.y / nz);
        for (int k = 0; k < nz; ++k) {
            const double2 v = col[k * st];
            col[k * st] = make_double2(v.x - shift.x, v.y - shift.y);
        }
        return;
    }
    const double sx = sin(M_PI * m / nx), sy = sin(M_PI * j / ny);
    const double b = 2.0 + 4.0 * (sx * sx + sy * sy);
    double c_prev = 0.0;
    double2 d_prev = make_double2(0.0, 0.0);
    for (int k = 0; k < nz; ++k) {
        const double2 r0 = col[k * st];
        const double2 r = make_double2(r0.x * scale, r0.y * scale);
        double diag = b;
        if (k == 0) diag -= s_lo;
        if (k == nz - 1) diag -= s_hi;
        const double den = (k == 0) ? diag : diag + c_prev;
        const double c = -1.0 / den;
        const double2 d = (k == 0) ? make_double2(r.x / den, r.y / den)
                                   : make_double2((r.x + d_prev.x) / den, (r.y + d_prev.y) / den);
        cpc[k * st] = c;
        col[k * st] = d;
        c_prev = c;
        d_prev = d;
    }
    double2 x = d_prev;
    for (int k = nz - 2; k >= 0; --k) {
        const double2 d = col[k * st];
        const double c = cpc[k * st];
        x = make_double2(d.x - c * x.x, d.y - c * x.y);
        col[k * st] = x;
    }
}

__global__ void zsolve_kernel(double2* __restrict__ spec, double* __restrict__ cp, int nx, int ny,
                              int nz, double scale, double s_lo, double s_hi, int singular,
                              int* __restrict__ flags) {
    const int nxh = nx / 2 + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nmode = nxh * ny;
    if (t >= nmode) return;
    zsolve_mode(spec + t, cp + t, (size_t)nmode, t % nxh, t / nxh, nx, ny, nz, scale, s_lo, s_hi,
                singular, flags);
}

// Batched: one thread per mode of every channel; mode_off is the prefix of the
// channels' mode counts (in mode_rep order).
__global__ void zsolve_batch_kernel(const RepDev* __restrict__ reps, const int* __restrict__ mode_off,
                                    const int* __restrict__ mode_rep, int nrep, int64_t nmode_tot,
                                    double2* __restrict__ spec, double* __restrict__ cp,
                                    int* __restrict__ flags) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nmode_tot) return;
    int lo = 0, hi = nrep - 1;  // last slot with mode_off[slot] <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (mode_off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const RepDev& R = reps[mode_rep[lo]];
    const int tl = (int)(t - mode_off[lo]);
    const int nxh = R.g.nxh;
    zsolve_mode(spec + R.spec_off + tl, cp + R.spec_off + tl, (size_t)R.nmode, tl % nxh, tl / nxh,
                R.g.nx, R.g.ny, R.g.nz, R.scale, R.s_lo, R.s_hi, R.singular, flags);
}

static int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Real FFT along x of nrows rows (nrows even) into half spectra, and its inverse;
// complex FFT along y of nlev levels of half spectra.
int fft_rows_r2c(Ctx* c, const double* in, double2* spec, int nrows, hipStream_t s) {
    const int nx = c->gd.nx;
    const int npairs = nrows / 2;
    const int ppb = std::max(1, 2048 / nx);
    fft_x_r2c_kernel<<<(npairs + ppb - 1) / ppb, FFT_THREADS, (size_t)ppb * nx * sizeof(double2), s>>>(
        in, spec, nx, ilog2(nx), npairs, ppb, c->tw_x);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int fft_rows_c2r(Ctx* c, const double2* spec, double* out, int nrows, hipStream_t s) {
    const int nx = c->gd.nx;
    const int npairs = nrows / 2;
    const int ppb = std::max(1, 2048 / nx);
    fft_x_c2r_kernel<<<(npairs + ppb - 1) / ppb, FFT_THREADS, (size_t)ppb * nx * sizeof(double2), s>>>(
        spec, out, nx, ilog2(nx), npairs, ppb, c->tw_x);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int fft_cols(Ctx* c, double2* spec, int nlev, int inv, hipStream_t s) {
    const int ny = c->gd.ny, nxh = c->gd.nxh;
    const int mc = std::max(1, std::min(16, 2048 / ny));
    dim3 gy((nxh + mc - 1) / mc, nlev);
    fft_y_kernel<<<gy, FFT_THREADS, (size_t)mc * ny * sizeof(double2), s>>>(spec, nxh, ny, ilog2(ny), mc,
                                                                           c->tw_y, inv);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int solve_poisson(Ctx* c, const double* rhs, const discos_params* p, double* phi, hipStream_t s,
                  int mark_base, int project) {
    const GridDev& g = c->gd;
    const int nx = g.nx, ny = g.ny, nz = g.nz, nxh = g.nxh;
    const int nrows = ny * nz;
    const int npairs = nrows / 2;
    const int ppb = std::max(1, 2048 / nx);
    const size_t ldsx = (size_t)ppb * nx * sizeof(double2);
    fft_x_r2c_kernel<<<(npairs + ppb - 1) / ppb, FFT_THREADS, ldsx, s>>>(rhs, c->spec, nx, ilog2(nx),
                                                                        npairs, ppb, c->tw_x);
    if (mark_base >= 0) stage_mark(c, mark_base, s);
    const int mc = std::max(1, std::min(16, 2048 / ny));
    const size_t ldsy = (size_t)mc * ny * sizeof(double2);
    dim3 gy((nxh + mc - 1) / mc, nz);
    fft_y_kernel<<<gy, FFT_THREADS, ldsy, s>>>(c->spec, nxh, ny, ilog2(ny), mc, c->tw_y, 0);
    if (mark_base >= 0) stage_mark(c, mark_base + 1, s);
    const double scale = (c->grid.h * c->grid.h / p->eps) / ((double)nx * ny);
    const double s_lo = p->bc_type[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    const double s_hi = p->bc_type[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    // 1: all-Neumann, check neutrality; 2: all-Neumann, pseudo-inverse of any rhs
    const int singular = (p->bc_type[0] == DISCOS_BC_NEUMANN && p->bc_type[1] == DISCOS_BC_NEUMANN)
                             ? (project ? 2 : 1)
                             : 0;
    const int nmode = nxh * ny;
    zsolve_kernel<<<(nmode + 63) / 64, 64, 0, s>>>(c->spec, c->cprime, nx, ny, nz, scale, s_lo, s_hi,
                                                  singular, c->flags);
    if (mark_base >= 0) stage_mark(c, mark_base + 2, s);
    fft_y_kernel<<<gy, FFT_THREADS, ldsy, s>>>(c->spec, nxh, ny, ilog2(ny), mc, c->tw_y, 1);
    if (mark_base >= 0) stage_mark(c, mark_base + 3, s);
    fft_x_c2r_kernel<<<(npairs + ppb - 1) / ppb, FFT_THREADS, ldsx, s>>>(c->spec, phi, nx, ilog2(nx),
                                                                        npairs, ppb, c->tw_x);
    if (mark_base >= 0) stage_mark(c, mark_base + 4, s);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

// Poisson for every channel: x- and y-FFTs per size class (a class's grids and spectra
// are contiguous, so its rows and levels form single ranges), one z-solve launch.
int batch_poisson(Batch* b, hipStream_t s) {
    for (const BatchClass& k : b->classes) {
        const int nxh = k.nx / 2 + 1;
        const int ppb = std::max(1, 2048 / k.nx);
        const int npairs = k.rows / 2;
        fft_x_r2c_kernel<<<(npairs + ppb - 1) / ppb, FFT_THREADS, (size_t)ppb * k.nx * sizeof(double2), s>>>(
            b->rho + k.cell_off, b->spec + k.spec_off, k.nx, ilog2(k.nx), npairs, ppb, k.tw_x);
        const int mc = std::max(1, std::min(16, 2048 / k.ny));
        dim3 gy((nxh + mc - 1) / mc, k.levels);
        fft_y_kernel<<<gy, FFT_THREADS, (size_t)mc * k.ny * sizeof(double2), s>>>(
            b->spec + k.spec_off, nxh, k.ny, ilog2(k.ny), mc, k.tw_y, 0);
    }
    zsolve_batch_kernel<<<(int)((b->nmode_tot + 63) / 64), 64, 0, s>>>(
        b->reps_d, b->mode_off, b->mode_rep, b->R, b->nmode_tot, b->spec, b->cprime, b->flags);
    for (const BatchClass& k : b->classes) {
        const int nxh = k.nx / 2 + 1;
        const int mc = std::max(1, std::min(16, 2048 / k.ny));
        dim3 gy((nxh + mc - 1) / mc, k.levels);
        fft_y_kernel<<<gy, FFT_THREADS, (size_t)mc * k.ny * sizeof(double2), s>>>(
            b->spec + k.spec_off, nxh, k.ny, ilog2(k.ny), mc, k.tw_y, 1);
        const int ppb = std::max(1, 2048 / k.nx);
        const int npairs = k.rows / 2;
        fft_x_c2r_kernel<<<(npairs + ppb - 1) / ppb, FFT_THREADS, (size_t)ppb * k.nx * sizeof(double2), s>>>(
            b->spec + k.spec_off, b->phi + k.cell_off, k.nx, ilog2(k.nx), npairs, ppb, k.tw_x);
    }
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
