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

// 1/a to full FP64 accuracy: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double recip(double a) {
    double y = __builtin_amdgcn_rcp(a);
    y = fma(fma(-a, y, 1.0), y, y);
    y = fma(fma(-a, y, 1.0), y, y);
    return y;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place radix-2 DIT FFTs of `lines` lines of length N = 2^logN stored back to back in
// LDS, input in bit-reversed order.  tw[k] = exp(-2 pi i k / N), k < N/2; `inv`
// conjugates.  Stages are taken two at a time (radix 2^2): a thread loads the four
// elements i, i+h, i+2h, i+3h of a group of 4h, applies stage s (pairs at distance h)
// and stage s+1 (pairs at distance 2h) in registers and stores once -- the same
// operations as two radix-2 stages, with half the LDS round trips and barriers.  An odd
// logN ends with one radix-2 stage.  Index arithmetic is shifts and masks.
__device__ void lds_fft(double2* a, int N, int logN, int lines, const double2* __restrict__ tw,
                        int inv) {
    const double sg = inv ? -1.0 : 1.0;
    int s = 1;
    if (logN >= 2) {
        const int lq = logN - 2;  // log2(N / 4)
        const int nq = lines << lq;
        for (; s + 1 <= logN; s += 2) {
            const int ls = s - 1;
            const int h = 1 << ls;
            for (int qd = threadIdx.x; qd < nq; qd += blockDim.x) {
                const int line = qd >> lq;
                const int qq = qd & ((1 << lq) - 1);
                const int grp = qq >> ls;
                const int p = qq & (h - 1);
                const int i0 = (line << logN) + (grp << (s + 1)) + p;
                double2 w1 = tw[p << (logN - s)];
                double2 wa = tw[p << (logN - s - 1)];
                double2 wb = tw[(p + h) << (logN - s - 1)];
                w1.y *= sg;
                wa.y *= sg;
                wb.y *= sg;
                const double2 x0 = a[i0], x1 = a[i0 + h], x2 = a[i0 + 2 * h], x3 = a[i0 + 3 * h];
                // stage s
                const double2 v1 = cmul(x1, w1), v3 = cmul(x3, w1);
                const double2 b0 = make_double2(x0.x + v1.x, x0.y + v1.y);
                const double2 b1 = make_double2(x0.x - v1.x, x0.y - v1.y);
                const double2 b2 = make_double2(x2.x + v3.x, x2.y + v3.y);
                const double2 b3 = make_double2(x2.x - v3.x, x2.y - v3.y);
                // stage s + 1
                const double2 c2 = cmul(b2, wa), c3 = cmul(b3, wb);
                a[i0] = make_double2(b0.x + c2.x, b0.y + c2.y);
                a[i0 + 2 * h] = make_double2(b0.x - c2.x, b0.y - c2.y);
                a[i0 + h] = make_double2(b1.x + c3.x, b1.y + c3.y);
                a[i0 + 3 * h] = make_double2(b1.x - c3.x, b1.y - c3.y);
            }
            __syncthreads();
        }
    }
    if (s == logN) {  // one radix-2 stage left
        const int lh = logN - 1;
        const int nb = lines << lh;
        const int ls = s - 1;
        const int half = 1 << ls;
        for (int bq = threadIdx.x; bq < nb; bq += blockDim.x) {
            const int line = bq >> lh;
            const int bb = bq & ((1 << lh) - 1);
            const int grp = bb >> ls;
            const int p = bb & (half - 1);
            const int i = (line << logN) + (grp << s) + p;
            const int j = i + half;
            double2 w = tw[p];
            w.y *= sg;
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
__device__ __forceinline__ void fft_x_r2c_block(const double* __restrict__ in, double2* __restrict__ spec,
                                                int nx, int logN, int npairs, int ppb,
                                                const double2* __restrict__ tw, int blk, double2* lds) {
    const int nxh = nx / 2 + 1;
    const int p0 = blk * ppb;
    for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
        const int p = e >> logN, n = e & (nx - 1);
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
    // e -> (p, m) with p = e / nxh through a float reciprocal (exact after one
    // correction for e < 2^20) instead of an integer division
    const float inv_nxh = 1.0f / (float)nxh;
    for (int e = threadIdx.x; e < ppb * nxh; e += blockDim.x) {
        int p = (int)((float)e * inv_nxh);
        int m = e - p * nxh;
        if (m < 0) {
            --p;
            m += nxh;
        } else if (m >= nxh) {
            ++p;
            m -= nxh;
        }
        const int pr = p0 + p;
        if (pr >= npairs) continue;
        const double2 Z = lds[p * nx + (m & (nx - 1))];
        const double2 Zr = lds[p * nx + ((nx - m) & (nx - 1))];
        // A = (Z + conj Zr) / 2, B = (Z - conj Zr) / (2i)
        const double2 A = make_double2(0.5 * (Z.x + Zr.x), 0.5 * (Z.y - Zr.y));
        const double2 B = make_double2(0.5 * (Z.y + Zr.y), -0.5 * (Z.x - Zr.x));
        const size_t r0 = 2 * (size_t)pr;
        spec[r0 * nxh + m] = A;
        spec[(r0 + 1) * nxh + m] = B;
    }
}

__global__ void __launch_bounds__(FFT_THREADS)
fft_x_r2c_kernel(const double* __restrict__ in, double2* __restrict__ spec, int nx, int logN,
                 int npairs, int ppb, const double2* __restrict__ tw) {
    extern __shared__ double2 lds[];
    fft_x_r2c_block(in, spec, nx, logN, npairs, ppb, tw, blockIdx.x, lds);
}

// Half spectra -> real rows (inverse, unnormalised).
__device__ __forceinline__ void fft_x_c2r_block(const double2* __restrict__ spec, double* __restrict__ out,
                                                int nx, int logN, int npairs, int ppb,
                                                const double2* __restrict__ tw, int blk, double2* lds) {
    const int nxh = nx / 2 + 1;
    const int p0 = blk * ppb;
    for (int e = threadIdx.x; e < ppb * nx; e += blockDim.x) {
        const int p = e >> logN, n = e & (nx - 1);
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
        const int p = e >> logN, n = e & (nx - 1);
        const int pr = p0 + p;
        if (pr >= npairs) continue;
        const size_t r0 = 2 * (size_t)pr;
        const double2 z = lds[p * nx + n];
        out[r0 * nx + n] = z.x;
        out[(r0 + 1) * nx + n] = z.y;
    }
}

__global__ void __launch_bounds__(FFT_THREADS)
fft_x_c2r_kernel(const double2* __restrict__ spec, double* __restrict__ out, int nx, int logN,
                 int npairs, int ppb, const double2* __restrict__ tw) {
    extern __shared__ double2 lds[];
    fft_x_c2r_block(spec, out, nx, logN, npairs, ppb, tw, blockIdx.x, lds);
}

// Complex FFTs along y of spec[k][j][m]: the columns (k, m) of nlev levels, numbered
// t = k nxh + m, are taken tpb at a time (tpb = 2^ltpb) by one block, so that no block
// holds padding columns and small grids put several levels in one block.  For a fixed j
// the block's columns are consecutive m (a level's boundary aside), so its loads and
// stores run along spectrum rows.
__device__ __forceinline__ void fft_y_block(double2* __restrict__ spec, int nxh, int ny, int logN,
                                            int ltpb, int ncol, const double2* __restrict__ tw,
                                            int inv, int blk, double2* lds) {
    const int tpb = 1 << ltpb;
    const int t0 = blk * tpb;
    // t -> (k, m) with k = t / nxh through a float reciprocal when t < 2^22 (t exact as a
    // float, the quotient off by at most one and corrected), else an integer division
    const float inv_nxh = 1.0f / (float)nxh;
    const bool fdiv = ncol < (1 << 22);
    auto at = [&](int t, int j) {
        int k = fdiv ? (int)((float)t * inv_nxh) : t / nxh;
        int m = t - k * nxh;
        if (m < 0) {
            --k;
            m += nxh;
        } else if (m >= nxh) {
            ++k;
            m -= nxh;
        }
        return ((size_t)k * ny + j) * nxh + m;
    };
    for (int e = threadIdx.x; e < tpb * ny; e += blockDim.x) {
        const int c = e & (tpb - 1), j = e >> ltpb;
        const int t = t0 + c;
        lds[c * ny + bitrev(j, logN)] = t < ncol ? spec[at(t, j)] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    lds_fft(lds, ny, logN, tpb, tw, inv);
    for (int e = threadIdx.x; e < tpb * ny; e += blockDim.x) {
        const int c = e & (tpb - 1), j = e >> ltpb;
        const int t = t0 + c;
        if (t < ncol) spec[at(t, j)] = lds[c * ny + j];
    }
}

__global__ void __launch_bounds__(FFT_THREADS)
fft_y_kernel(double2* __restrict__ spec, int nxh, int ny, int logN, int ltpb, int ncol,
             const double2* __restrict__ tw, int inv) {
    extern __shared__ double2 lds[];
    // consecutive blocks (neighbouring columns, which share cache lines) on one XCD
    fft_y_block(spec, nxh, ny, logN, ltpb, ncol, tw, inv, xcd_block(blockIdx.x, gridDim.x), lds);
}

// The same passes over every (nx, ny) class of a batch in one launch: block b belongs
// to the last class whose first block (xb0 for the x passes, yb0 for the y pass) is at
// most b.
__device__ __forceinline__ int fft_class_of(const FftClassDev* __restrict__ cls, int ncls, int b, bool y) {
    int k = 0;
    while (k + 1 < ncls && (y ? cls[k + 1].yb0 : cls[k + 1].xb0) <= b) ++k;
    return k;
}

__global__ void __launch_bounds__(FFT_THREADS)
fft_x_r2c_cls_kernel(const FftClassDev* __restrict__ cls, int ncls, const double* __restrict__ in,
                     double2* __restrict__ spec) {
    extern __shared__ double2 lds[];
    const int k = fft_class_of(cls, ncls, blockIdx.x, false);
    const FftClassDev& c = cls[k];
    fft_x_r2c_block(in + c.cell_off, spec + c.spec_off, c.nx, c.logx, c.npairs, c.ppb, c.tw_x,
                    blockIdx.x - c.xb0, lds);
}

__global__ void __launch_bounds__(FFT_THREADS)
fft_x_c2r_cls_kernel(const FftClassDev* __restrict__ cls, int ncls, const double2* __restrict__ spec,
                     double* __restrict__ out) {
    extern __shared__ double2 lds[];
    const int k = fft_class_of(cls, ncls, blockIdx.x, false);
    const FftClassDev& c = cls[k];
    fft_x_c2r_block(spec + c.spec_off, out + c.cell_off, c.nx, c.logx, c.npairs, c.ppb, c.tw_x,
                    blockIdx.x - c.xb0, lds);
}

__global__ void __launch_bounds__(FFT_THREADS)
fft_y_cls_kernel(const FftClassDev* __restrict__ cls, int ncls, double2* __restrict__ spec, int inv) {
    extern __shared__ double2 lds[];
    const int b = xcd_block(blockIdx.x, gridDim.x);  // a class's levels on neighbouring XCDs
    const int k = fft_class_of(cls, ncls, b, true);
    const FftClassDev& c = cls[k];
    fft_y_block(spec + c.spec_off, c.nxh, c.ny, c.logy, c.ltpb, c.ncol, c.tw_y, inv, b - c.yb0, lds);
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
    // Forward sweep.  Whole windows of ZW levels are fetched before use (no bounds test
    // inside a window, so all ZW loads are in flight together: a thread per mode leaves
    // few wavefronts, and only outstanding loads hide the memory latency); the last
    // nz % ZW levels go one by one.  One reciprocal per level (hardware estimate + two
    // Newton steps).
    constexpr int ZW = 16;
    double c_prev = 0.0;
    double2 d_prev = make_double2(0.0, 0.0);
    auto fwd = [&](int k, double2 rk) {
        double diag = b;
        if (k == 0) diag -= s_lo;
        if (k == nz - 1) diag -= s_hi;
        const double den = (k == 0) ? diag : diag + c_prev;
        const double inv = recip(den);
        const double2 d = make_double2((rk.x * scale + d_prev.x) * inv, (rk.y * scale + d_prev.y) * inv);
        cpc[(size_t)k * st] = -inv;
        col[(size_t)k * st] = d;
        c_prev = -inv;
        d_prev = d;
    };
    int k0 = 0;
    for (; k0 + ZW <= nz; k0 += ZW) {
        double2 rb[ZW];
#pragma unroll
        for (int u = 0; u < ZW; ++u) rb[u] = col[(size_t)(k0 + u) * st];
#pragma unroll
        for (int u = 0; u < ZW; ++u) fwd(k0 + u, rb[u]);
    }
    for (; k0 < nz; ++k0) fwd(k0, col[(size_t)k0 * st]);
    // back substitution over levels nz-2 .. 0, likewise by whole windows
    double2 x = d_prev;
    int k1 = nz - 2;
    for (; k1 - ZW + 1 >= 0; k1 -= ZW) {
        double2 db[ZW];
        double cb[ZW];
#pragma unroll
        for (int u = 0; u < ZW; ++u) {
            db[u] = col[(size_t)(k1 - u) * st];
            cb[u] = cpc[(size_t)(k1 - u) * st];
        }
#pragma unroll
        for (int u = 0; u < ZW; ++u) {
            x = make_double2(db[u].x - cb[u] * x.x, db[u].y - cb[u] * x.y);
            col[(size_t)(k1 - u) * st] = x;
        }
    }
    for (; k1 >= 0; --k1) {
        const double2 d = col[(size_t)k1 * st];
        const double c = cpc[(size_t)k1 * st];
        x = make_double2(d.x - c * x.x, d.y - c * x.y);
        col[(size_t)k1 * st] = x;
    }
}

__global__ void __launch_bounds__(64) zsolve_kernel(double2* __restrict__ spec, double* __restrict__ cp, int nx, int ny,
                              int nz, double scale, double s_lo, double s_hi, int singular,
                              int* __restrict__ flags) {
    const int nxh = nx / 2 + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nmode = nxh * ny;
    if (t >= nmode) return;
    zsolve_mode(spec + t, cp + t, (size_t)nmode, t % nxh, t / nxh, nx, ny, nz, scale, s_lo, s_hi,
                singular, flags);
}

// Batched, for channels with nz > 128: one thread per mode of every channel; mode_off
// is the prefix of the channels' mode counts (in mode_rep order).
__global__ void __launch_bounds__(64) zsolve_batch_kernel(const RepDev* __restrict__ reps, const int* __restrict__ mode_off,
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
    if (R.g.nz <= 128) return;  // solved with pivots
    const int tl = (int)(t - mode_off[lo]);
    const int nxh = R.g.nxh;
    zsolve_mode(spec + R.spec_off + tl, cp + R.spec_off + tl, (size_t)R.nmode, tl % nxh, tl / nxh,
                R.g.nx, R.g.ny, R.g.nz, R.scale, R.s_lo, R.s_hi, R.singular, flags);
}

// Pivots of the per-mode Thomas factorisation, g_k = 1 / (diag_k - g_{k-1}) (the
// reciprocal pivots; RHS independent), for every mode: [nz][nmode].  The singular
// kappa = 0 mode of an all-Neumann problem is solved separately and gets none.
__global__ void __launch_bounds__(64) zpivot_kernel(double* __restrict__ zg, int nx, int ny, int nz,
                                                   double s_lo, double s_hi, int singular) {
    const int nxh = nx / 2 + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nmode = nxh * ny;
    if (t >= nmode) return;
    const int m = t % nxh, j = t / nxh;
    const double sx = sin(M_PI * m / nx), sy = sin(M_PI * j / ny);
    const double b = 2.0 + 4.0 * (sx * sx + sy * sy);
    double gprev = 0.0;
    for (int k = 0; k < nz; ++k) {
        double diag = b;
        if (k == 0) diag -= s_lo;
        if (k == nz - 1) diag -= s_hi;
        const double gk = (singular && t == 0) ? 0.0 : recip(diag - gprev);
        zg[(size_t)k * nmode + t] = gk;
        gprev = gk;
    }
}

// Solve along z with the pivots g: forward d_k = g_k (r_k + d_{k-1}), back
// x_k = d_k + g_k x_{k+1} (x_nz = 0) -- two first-order linear recurrences.  S lanes
// share a mode, each holding one segment of L levels in registers: a segment's local
// recurrence gives an affine map (product of its g, local end value), a scan of those
// maps over the S lanes gives each segment's carry, and a second pass applies it.
// Lane l of a wavefront: mode M w + (l mod M), segment l / M with M = 64 / S, so one load
// instruction reads M consecutive modes at S levels.
template <int L, int S = 4>
__device__ __forceinline__ void zsolve_seg_wave(double2* __restrict__ spec, const double* __restrict__ zg,
                                                int nmode, int nz, double scale, int skip0, int t0) {
    static_assert(S == 4 || S == 8 || S == 16, "segments per mode");
    constexpr int ML = 64 / S;  // modes per wavefront
    const int lane = threadIdx.x & 63;
    const int ml = lane % ML, seg = lane / ML;
    const int t = t0 + ml;
    const bool valid = t < nmode && !(skip0 && t == 0);
    const int tt = min(t, nmode - 1);
    const int k0 = seg * L;
    const int len = max(0, min(L, nz - k0));
    double2 d[L];
    double g[L];
#pragma unroll
    for (int u = 0; u < L; ++u) {
        const size_t k = (size_t)min(k0 + u, nz - 1);
        d[u] = spec[k * nmode + tt];
        g[u] = zg[k * nmode + tt];
    }
    // forward, local (carry in = 0)
    double2 dl = make_double2(0.0, 0.0);
    double A = 1.0;
#pragma unroll
    for (int u = 0; u < L; ++u) {
        if (u < len) {
            dl = make_double2(g[u] * (d[u].x * scale + dl.x), g[u] * (d[u].y * scale + dl.y));
            A *= g[u];
            d[u] = dl;
        }
    }
    // carry into this segment: the affine maps x -> A x + dl of the segments below,
    // composed by an inclusive scan over the segments (log2 S rounds), then shifted by one
    double Ac = A, cx = dl.x, cy = dl.y;
#pragma unroll
    for (int o = 1; o < S; o <<= 1) {
        const double Ap = __shfl_up(Ac, ML * o, 64);
        const double px = __shfl_up(cx, ML * o, 64), py = __shfl_up(cy, ML * o, 64);
        if (seg >= o) {
            cx = Ac * px + cx;
            cy = Ac * py + cy;
            Ac *= Ap;
        }
    }
    const double cinx = __shfl_up(cx, ML, 64), ciny = __shfl_up(cy, ML, 64);
    const double2 din = seg > 0 ? make_double2(cinx, ciny) : make_double2(0.0, 0.0);
    double p = 1.0;
#pragma unroll
    for (int u = 0; u < L; ++u) {
        if (u < len) {
            p *= g[u];
            d[u] = make_double2(d[u].x + p * din.x, d[u].y + p * din.y);
        }
    }
    // backward, local (x at the segment's top boundary = 0)
    double2 xl = make_double2(0.0, 0.0);
    double B = 1.0;
#pragma unroll
    for (int u = L - 1; u >= 0; --u) {
        if (u < len) {
            xl = make_double2(d[u].x + g[u] * xl.x, d[u].y + g[u] * xl.y);
            B *= g[u];
            d[u] = xl;
        }
    }
    // the segments above, composed from the top down the same way
    double Bc = B, ex = xl.x, ey = xl.y;
#pragma unroll
    for (int o = 1; o < S; o <<= 1) {
        const double Bn = __shfl_down(Bc, ML * o, 64);
        const double nx = __shfl_down(ex, ML * o, 64), ny = __shfl_down(ey, ML * o, 64);
        if (seg + o < S) {
            ex = Bc * nx + ex;
            ey = Bc * ny + ey;
            Bc *= Bn;
        }
    }
    const double xinx = __shfl_down(ex, ML, 64), xiny = __shfl_down(ey, ML, 64);
    const double2 xin = seg + 1 < S ? make_double2(xinx, xiny) : make_double2(0.0, 0.0);
    double q = 1.0;
#pragma unroll
    for (int u = L - 1; u >= 0; --u) {
        if (u < len) {
            q *= g[u];
            d[u] = make_double2(d[u].x + q * xin.x, d[u].y + q * xin.y);
        }
    }
    if (!valid) return;
#pragma unroll
    for (int u = 0; u < L; ++u)
        if (u < len) spec[(size_t)(k0 + u) * nmode + t] = d[u];
}

__device__ __forceinline__ void zsolve_mode0_wave(double2* __restrict__ spec, int nmode, int nz,
                                                  double scale, int singular, int* __restrict__ flags);

// Wavefront w of block b solves modes M (4 b + w) .. + M - 1, M = 64 / S, each mode in S
// segments of L levels.  With singular != 0 mode 0 is skipped there and solved by the
// first wavefront of one extra last block.
template <int L, int S>
__global__ void __launch_bounds__(256) zsolve_seg_kernel(double2* __restrict__ spec,
                                                        const double* __restrict__ zg, int nmode,
                                                        int nz, double scale, int singular,
                                                        int* __restrict__ flags) {
    if (singular && blockIdx.x == gridDim.x - 1) {
        if (threadIdx.x < 64) zsolve_mode0_wave(spec, nmode, nz, scale, singular, flags);
        return;
    }
    zsolve_seg_wave<L, S>(spec, zg, nmode, nz, scale, singular != 0,
                          (blockIdx.x * 4 + (threadIdx.x >> 6)) * (64 / S));
}

// Batched: task (channel, first mode) per wavefront, for channels whose nz fits L
// levels per segment; the pivots of each channel's grid shape start at zg_off.
template <int L>
__global__ void __launch_bounds__(256) zsolve_seg_batch_kernel(const RepDev* __restrict__ reps,
                                                              const int2* __restrict__ tasks,
                                                              int ntasks, double2* __restrict__ spec,
                                                              const double* __restrict__ zg) {
    const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (task >= ntasks) return;  // the whole wavefront
    const int2 tk = tasks[task];
    const RepDev& R = reps[tk.x];
    zsolve_seg_wave<L>(spec + R.spec_off, zg + R.zg_off, R.nmode, R.g.nz, R.scale, R.singular != 0,
                       tk.y);
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_incl_scan(double v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// The singular kappa = 0 mode of an all-Neumann problem, by one wavefront.  Its rows
// (x_0 - x_1 = r_0, -x_{k-1} + 2 x_k - x_{k+1} = r_k, -x_{nz-2} + x_{nz-1} = r_{nz-1})
// are solvable iff sum r = 0 (neutrality; flagged unless the caller asked for the
// pseudo-inverse); with r' = r - mean(r) the differences are
// x_{k+1} - x_k = -(r'_0 + ... + r'_k), so x is a double prefix sum, shifted to mean 0:
// the minimum-norm solution.  Levels are taken 64 at a time with running carries.
__device__ __forceinline__ void zsolve_mode0_wave(double2* __restrict__ spec, int nmode, int nz,
                                                  double scale, int singular, int* __restrict__ flags) {
    const int lane = threadIdx.x & 63;
    double sx = 0.0, sy = 0.0, ax = 0.0;
    for (int k0 = 0; k0 < nz; k0 += 64) {
        const int k = k0 + lane;
        if (k < nz) {
            const double2 r = spec[(size_t)k * nmode];
            sx += r.x;
            sy += r.y;
            ax += sqrt(r.x * r.x + r.y * r.y);
        }
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    ax = wave_sum(ax);
    if (lane == 0 && singular == 1 && sqrt(sx * sx + sy * sy) > 1e-10 * fmax(ax, 1e-300))
        set_flag(flags, DISCOS_FLAG_NOT_NEUTRAL);
    const double mx = sx / nz, my = sy / nz;
    // pass 1: x_k (with x_0 = 0) = sum_{m<k} D_m, D_m = -S_m, S_m = r'_0 + .. + r'_m
    double cSx = 0.0, cSy = 0.0, cXx = 0.0, cXy = 0.0, tx = 0.0, ty = 0.0;
    for (int k0 = 0; k0 < nz; k0 += 64) {
        const int k = k0 + lane;
        double2 r = make_double2(0.0, 0.0);
        if (k < nz) r = spec[(size_t)k * nmode];
        const double rx = (k < nz) ? (r.x - mx) * scale : 0.0;
        const double ry = (k < nz) ? (r.y - my) * scale : 0.0;
        const double Sx = wave_incl_scan(rx) + cSx, Sy = wave_incl_scan(ry) + cSy;
        // x_k = -(S_0 + .. + S_{k-1}): exclusive scan of S
        const double Ix = wave_incl_scan(Sx), Iy = wave_incl_scan(Sy);
        const double xx = -(Ix - Sx + cXx), xy = -(Iy - Sy + cXy);
        if (k < nz) {
            spec[(size_t)k * nmode] = make_double2(xx, xy);
            tx += xx;
            ty += xy;
        }
        cSx = __shfl(Sx, 63, 64);
        cSy = __shfl(Sy, 63, 64);
        cXx += __shfl(Ix, 63, 64);
        cXy += __shfl(Iy, 63, 64);
    }
    // pass 2: mean zero
    tx = wave_sum(tx) / nz;
    ty = wave_sum(ty) / nz;
    for (int k0 = 0; k0 < nz; k0 += 64) {
        const int k = k0 + lane;
        if (k < nz) {
            const double2 v = spec[(size_t)k * nmode];
            spec[(size_t)k * nmode] = make_double2(v.x - tx, v.y - ty);
        }
    }
}

// Batched: block r solves the kappa = 0 mode of channel r when its walls are both
// Neumann and its z-solve uses pivots (nz <= 128).
__global__ void __launch_bounds__(64) zsolve_mode0_batch_kernel(const RepDev* __restrict__ reps,
                                                               double2* __restrict__ spec,
                                                               int* __restrict__ flags) {
    const RepDev& R = reps[blockIdx.x];
    if (!R.singular || R.g.nz > 128) return;
    zsolve_mode0_wave(spec + R.spec_off, R.nmode, R.g.nz, R.scale, R.singular, flags);
}

static int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Launch shape of the x passes over npairs row pairs: 512 elements (512 / nx pairs) per
// block, four per thread.  (The y pass takes 1024 per block: its blocks read spectrum
// rows column-wise, and wider blocks read longer runs of each row.)
#define FFT_X_POINTS 512
struct XLaunch {
    int ppb, threads, blocks;
    size_t lds;
};
static XLaunch x_launch(int nx, int npairs) {
    XLaunch L;
    L.ppb = std::max(1, FFT_X_POINTS / nx);
    L.threads = std::min(FFT_THREADS, std::max(64, L.ppb * nx / 4));
    L.blocks = (npairs + L.ppb - 1) / L.ppb;
    L.lds = (size_t)L.ppb * nx * sizeof(double2);
    return L;
}

// Real FFT along x of nrows rows (nrows even) into half spectra, and its inverse;
// complex FFT along y of nlev levels of half spectra.
int fft_rows_r2c(Ctx* c, const double* in, double2* spec, int nrows, hipStream_t s) {
    const int nx = c->gd.nx;
    const int npairs = nrows / 2;
    const XLaunch X = x_launch(nx, npairs);
    fft_x_r2c_kernel<<<X.blocks, X.threads, X.lds, s>>>(in, spec, nx, ilog2(nx), npairs, X.ppb,
                                                        c->tw_x);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int fft_rows_c2r(Ctx* c, const double2* spec, double* out, int nrows, hipStream_t s) {
    const int nx = c->gd.nx;
    const int npairs = nrows / 2;
    const XLaunch X = x_launch(nx, npairs);
    fft_x_c2r_kernel<<<X.blocks, X.threads, X.lds, s>>>(spec, out, nx, ilog2(nx), npairs, X.ppb,
                                                        c->tw_x);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

// The y pass over nlev levels: 1024 elements (1024 / ny columns) per block.
static void fft_y_launch(const Ctx* c, double2* spec, int nlev, int inv, hipStream_t s) {
    const int ny = c->gd.ny, nxh = c->gd.nxh;
    const int ltpb = ilog2(std::max(1, 1024 / ny));
    const int ncol = nlev * nxh;
    fft_y_kernel<<<(ncol + (1 << ltpb) - 1) >> ltpb, FFT_THREADS, ((size_t)ny << ltpb) * sizeof(double2),
                   s>>>(spec, nxh, ny, ilog2(ny), ltpb, ncol, c->tw_y, inv);
}

// out = F^-1 [C_k F in] on a pair of (x, y) planes (in, out: [2][ny][nx]; spectra in
// c->spec): per in-plane mode k the 2 x 2 symmetric map C_k = [[c0, c1], [c1, c2]]
// (coef: [3][ny][nx/2 + 1]) couples the two planes' coefficients; out includes the
// 1 / (nx ny) of the inverse transforms.
__global__ void plane_pair_mode_kernel(int nmode, double2* __restrict__ spec,
                                       const double* __restrict__ coef, double norm) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nmode) return;
    const double c0 = coef[t] * norm, c1 = coef[nmode + t] * norm, c2 = coef[2 * nmode + t] * norm;
    const double2 a = spec[t], b = spec[nmode + t];
    spec[t] = make_double2(c0 * a.x + c1 * b.x, c0 * a.y + c1 * b.y);
    spec[nmode + t] = make_double2(c1 * a.x + c2 * b.x, c1 * a.y + c2 * b.y);
}

int plane_pair_filter(Ctx* c, const double* in, double* out, const double* coef, hipStream_t s) {
    const GridDev& g = c->gd;
    const int nx = g.nx, ny = g.ny, nxh = g.nxh;
    const int npairs = ny;  // 2 ny rows
    const XLaunch X = x_launch(nx, npairs);
    fft_x_r2c_kernel<<<X.blocks, X.threads, X.lds, s>>>(in, c->spec, nx, ilog2(nx), npairs, X.ppb,
                                                        c->tw_x);
    fft_y_launch(c, c->spec, 2, 0, s);
    const int nmode = nxh * ny;
    plane_pair_mode_kernel<<<(nmode + 255) / 256, 256, 0, s>>>(nmode, c->spec, coef,
                                                                1.0 / ((double)nx * ny));
    fft_y_launch(c, c->spec, 2, 1, s);
    fft_x_c2r_kernel<<<X.blocks, X.threads, X.lds, s>>>(c->spec, out, nx, ilog2(nx), npairs, X.ppb,
                                                        c->tw_x);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int fft_cols(Ctx* c, double2* spec, int nlev, int inv, hipStream_t s) {
    fft_y_launch(c, spec, nlev, inv, s);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

int solve_poisson(Ctx* c, const double* rhs, const discos_params* p, double* phi, hipStream_t s,
                  int mark_base, int project) {
    if (c->wm_mixed && (p->bc_type_map[0] || p->bc_type_map[1])) {
        // walls of mixed type: the iterative solve (timed whole as the first stage)
        const int rc = solve_poisson_mixed(c, rhs, p, c->wm_ref, phi, s);
        if (mark_base >= 0)
            for (int k = 0; k < 5; ++k) stage_mark(c, mark_base + k, s);
        return rc;
    }
    const GridDev& g = c->gd;
    const int nx = g.nx, ny = g.ny, nz = g.nz, nxh = g.nxh;
    const int nrows = ny * nz;
    const int npairs = nrows / 2;
    const XLaunch X = x_launch(nx, npairs);
    fft_x_r2c_kernel<<<X.blocks, X.threads, X.lds, s>>>(rhs, c->spec, nx, ilog2(nx), npairs, X.ppb,
                                                        c->tw_x);
    if (mark_base >= 0) stage_mark(c, mark_base, s);
    fft_y_launch(c, c->spec, nz, 0, s);
    if (mark_base >= 0) stage_mark(c, mark_base + 1, s);
    const double scale = (c->grid.h * c->grid.h / p->eps) / ((double)nx * ny);
    const double s_lo = p->bc_type[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    const double s_hi = p->bc_type[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    // 1: all-Neumann, check neutrality; 2: all-Neumann, pseudo-inverse of any rhs
    const int singular = (p->bc_type[0] == DISCOS_BC_NEUMANN && p->bc_type[1] == DISCOS_BC_NEUMANN)
                             ? (project ? 2 : 1)
                             : 0;
    const int nmode = nxh * ny;
    if (nz <= 128) {
        // pivots once per wall-type pair (the buffer then holds them, not Thomas scratch)
        const int key = p->bc_type[0] * 2 + p->bc_type[1];
        if (c->zg_key != key) {
            zpivot_kernel<<<(nmode + 63) / 64, 64, 0, s>>>(c->cprime, nx, ny, nz, s_lo, s_hi, singular != 0);
            c->zg_key = key;
        }
        // segments of 8 levels, 4, 8 or 16 per mode: few registers per wavefront (about 80),
        // so that the solve's wavefronts find room beside other work on the device
        const int S = nz <= 32 ? 4 : nz <= 64 ? 8 : 16;
        const int per_block = 4 * (64 / S);
        // one extra block carries the singular kappa = 0 mode
        const int nb = (nmode + per_block - 1) / per_block + (singular ? 1 : 0);
        if (S == 4)
            zsolve_seg_kernel<8, 4><<<nb, 256, 0, s>>>(c->spec, c->cprime, nmode, nz, scale, singular, c->flags);
        else if (S == 8)
            zsolve_seg_kernel<8, 8><<<nb, 256, 0, s>>>(c->spec, c->cprime, nmode, nz, scale, singular, c->flags);
        else
            zsolve_seg_kernel<8, 16><<<nb, 256, 0, s>>>(c->spec, c->cprime, nmode, nz, scale, singular, c->flags);
    } else {
        c->zg_key = -1;
        zsolve_kernel<<<(nmode + 63) / 64, 64, 0, s>>>(c->spec, c->cprime, nx, ny, nz, scale, s_lo, s_hi,
                                                      singular, c->flags);
    }
    if (mark_base >= 0) stage_mark(c, mark_base + 2, s);
    fft_y_launch(c, c->spec, nz, 1, s);
    if (mark_base >= 0) stage_mark(c, mark_base + 3, s);
    fft_x_c2r_kernel<<<X.blocks, X.threads, X.lds, s>>>(c->spec, phi, nx, ilog2(nx), npairs, X.ppb,
                                                        c->tw_x);
    if (mark_base >= 0) stage_mark(c, mark_base + 4, s);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

// Pivots of every grid shape of a batch with nz <= 128 (all channels share the wall types).
int batch_pivots(Batch* b, hipStream_t s) {
    const double s_lo = b->p.bc_type[0] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    const double s_hi = b->p.bc_type[1] == DISCOS_BC_DIRICHLET ? -1.0 : 1.0;
    for (const auto& sh : b->zshapes) {
        const int nx = (int)sh[0], ny = (int)sh[1], nz = (int)sh[2];
        const int nmode = (nx / 2 + 1) * ny;
        zpivot_kernel<<<(nmode + 63) / 64, 64, 0, s>>>(b->zg + sh[3], nx, ny, nz, s_lo, s_hi,
                                                        b->z_singular ? 1 : 0);
    }
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

// Poisson for every channel: each FFT pass one launch over every (nx, ny) class (a
// class's grids and spectra are contiguous, so its rows and levels form single ranges);
// z-solves with pivots per segment length (one launch each), the Thomas sweep for
// channels with nz > 128.
int batch_poisson(Batch* b, hipStream_t s) {
    const int ncls = (int)b->classes.size();
    fft_x_r2c_cls_kernel<<<b->fft_xblocks, FFT_THREADS, b->fft_xlds, s>>>(b->fcls, ncls, b->rho, b->spec);
    fft_y_cls_kernel<<<b->fft_yblocks, FFT_THREADS, b->fft_ylds, s>>>(b->fcls, ncls, b->spec, 0);
    if (b->ztasks_n[0] > 0)
        zsolve_seg_batch_kernel<8><<<(b->ztasks_n[0] + 3) / 4, 256, 0, s>>>(b->reps_d, b->ztasks[0],
                                                                          b->ztasks_n[0], b->spec, b->zg);
    if (b->ztasks_n[1] > 0)
        zsolve_seg_batch_kernel<16><<<(b->ztasks_n[1] + 3) / 4, 256, 0, s>>>(b->reps_d, b->ztasks[1],
                                                                           b->ztasks_n[1], b->spec, b->zg);
    if (b->ztasks_n[2] > 0)
        zsolve_seg_batch_kernel<32><<<(b->ztasks_n[2] + 3) / 4, 256, 0, s>>>(b->reps_d, b->ztasks[2],
                                                                           b->ztasks_n[2], b->spec, b->zg);
    if (b->z_singular) zsolve_mode0_batch_kernel<<<b->R, 64, 0, s>>>(b->reps_d, b->spec, b->flags);
    if (b->z_legacy)
        zsolve_batch_kernel<<<(int)((b->nmode_tot + 63) / 64), 64, 0, s>>>(
            b->reps_d, b->mode_off, b->mode_rep, b->R, b->nmode_tot, b->spec, b->cprime, b->flags);
    fft_y_cls_kernel<<<b->fft_yblocks, FFT_THREADS, b->fft_ylds, s>>>(b->fcls, ncls, b->spec, 1);
    fft_x_c2r_cls_kernel<<<b->fft_xblocks, FFT_THREADS, b->fft_xlds, s>>>(b->fcls, ncls, b->spec, b->phi);
    return hipGetLastError() == hipSuccess ? DISCOS_OK : DISCOS_E_HIP;
}

}  // namespace discos
