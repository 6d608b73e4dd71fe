// The grid pair-force table of the P3M near-field correction (Sec. II.B.1, eq LC): the
// radial field that the grid operators produce between two charges, measured the way
// the paper describes.  A unit charge is spread with the 4-point Peskin kernel (eq
// peskin1d) onto a triply periodic n^3 box of unit cells, the Poisson problem with the
// 7-point Laplacian and eps = 1 / (4 pi) is solved by FFT in the zero-mean gauge, the
// face differences E = -grad_h phi are interpolated back at distance rho along a given
// direction, the neutralising background's field rho / (3 eps V) is removed, and the
// radial component is averaged over the placements.  Host code, run once per table.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "discos.h"

namespace {

using cplx = std::complex<double>;

// In-place radix-2 transform of n points spaced s apart; tw[k] = exp(-2 pi i k / n).
// Forward (inverse = false) is sum_j a_j exp(-2 pi i j k / n); the inverse is unscaled.
void fft_line(cplx* a, int n, int s, bool inverse, const std::vector<cplx>& tw) {
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[(size_t)i * s], a[(size_t)j * s]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len / 2, step = n / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < half; ++k) {
                const cplx w = inverse ? std::conj(tw[(size_t)k * step]) : tw[(size_t)k * step];
                cplx& lo = a[(size_t)(i + k) * s];
                cplx& hi = a[(size_t)(i + k + half) * s];
                const cplx v = hi * w;
                hi = lo - v;
                lo = lo + v;
            }
    }
}

// 3-D transform of an n^3 array laid out [z][y][x].
void fft_box(std::vector<cplx>& a, int n, bool inverse, const std::vector<cplx>& tw) {
    const size_t n2 = (size_t)n * n;
    for (size_t zy = 0; zy < n2; ++zy) fft_line(&a[zy * n], n, 1, inverse, tw);
    for (int z = 0; z < n; ++z)
        for (int x = 0; x < n; ++x) fft_line(&a[z * n2 + x], n, n, inverse, tw);
    for (size_t yx = 0; yx < n2; ++yx) fft_line(&a[yx], n, (int)n2, inverse, tw);
}

// 4-point Peskin kernel (eq peskin1d) at r cells.
double peskin(double r) {
    r = std::fabs(r);
    if (r < 1.0) return (3.0 - 2.0 * r + std::sqrt(1.0 + 4.0 * r - 4.0 * r * r)) * 0.125;
    if (r < 2.0) return (5.0 - 2.0 * r - std::sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) * 0.125;
    return 0.0;
}

// Nodes floor(s) - 1 .. floor(s) + 2 (wrapped into [0, n)) and their kernel weights.
void axis_weights(double s, int n, int idx[4], double w[4]) {
    const double f = std::floor(s);
    for (int a = 0; a < 4; ++a) {
        const double node = f - 1.0 + a;
        w[a] = peskin(s - node);
        int k = (int)node % n;
        idx[a] = k < 0 ? k + n : k;
    }
}

double wrap(double x, double L) {
    double r = std::fmod(x, L);
    if (r < 0.0) r += L;
    return r >= L ? 0.0 : r;
}

// Radial field at distances k * drho (k < nrho) from one unit charge at src, along the
// directions dir[3][nrho] (normalised here), background term removed.
void one_placement(int n, int nrho, double drho, const double* src, const double* dir,
                   const std::vector<cplx>& tw, const std::vector<double>& inv_k2, double* out) {
    const size_t n2 = (size_t)n * n, n3 = n2 * n;
    const double eps = 1.0 / (4.0 * M_PI);
    const double L = (double)n;
    std::vector<cplx> a(n3, cplx(0.0, 0.0));
    // spread: cell centres sit at (i + 1/2) h
    int ix[4], iy[4], iz[4];
    double wx[4], wy[4], wz[4];
    axis_weights(src[0] - 0.5, n, ix, wx);
    axis_weights(src[1] - 0.5, n, iy, wy);
    axis_weights(src[2] - 0.5, n, iz, wz);
    for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
            for (int d = 0; d < 4; ++d)
                a[(size_t)iz[c] * n2 + (size_t)iy[b] * n + ix[d]] += wx[d] * wy[b] * wz[c];
    // -eps lap_h phi = rho, zero mean
    fft_box(a, n, false, tw);
    for (size_t k = 0; k < n3; ++k) a[k] *= inv_k2[k] / eps;
    fft_box(a, n, true, tw);
    std::vector<double> phi(n3);
    for (size_t k = 0; k < n3; ++k) phi[k] = a[k].real() / (double)n3;
    auto at = [&](int z, int y, int x) { return phi[(size_t)z * n2 + (size_t)y * n + x]; };
    const double bg = 1.0 / (3.0 * eps * (double)n3);
    for (int k = 0; k < nrho; ++k) {
        const double rho = k * drho;
        double u[3] = {dir[k], dir[nrho + k], dir[2 * nrho + k]};
        const double nu = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        for (double& v : u) v /= nu;
        double t[3];
        for (int d = 0; d < 3; ++d) t[d] = wrap(src[d] + rho * u[d], L);
        double radial = 0.0;
        for (int comp = 0; comp < 3; ++comp) {
            // E_comp lives on the faces normal to comp: offset 0 along comp, 1/2 across
            axis_weights(t[0] - (comp == 0 ? 0.0 : 0.5), n, ix, wx);
            axis_weights(t[1] - (comp == 1 ? 0.0 : 0.5), n, iy, wy);
            axis_weights(t[2] - (comp == 2 ? 0.0 : 0.5), n, iz, wz);
            double e = 0.0;
            for (int c = 0; c < 4; ++c)
                for (int b = 0; b < 4; ++b)
                    for (int d = 0; d < 4; ++d) {
                        const int x = ix[d], y = iy[b], z = iz[c];
                        // face F between cells F - 1 and F: E = -(phi_F - phi_{F-1}) / h
                        const double lo = comp == 0 ? at(z, y, (x + n - 1) % n)
                                        : comp == 1 ? at(z, (y + n - 1) % n, x)
                                                    : at((z + n - 1) % n, y, x);
                        e += wx[d] * wy[b] * wz[c] * -(at(z, y, x) - lo);
                    }
            radial += e * u[comp];
        }
        out[k] = radial + rho * bg;
    }
}

}  // namespace

extern "C" int discos_p3m_table(int n, int nplace, int nrho, double drho, const double* src,
                                const double* dir, double* g) {
    if (n < 8 || n > 256 || (n & (n - 1)) || nplace < 1 || nrho < 1 || !(drho > 0.0) ||
        !std::isfinite(drho) || !src || !dir || !g)
        return DISCOS_E_ARG;
    // no exception may leave this function: allocation failures become an error code
    try {
        const size_t n2 = (size_t)n * n, n3 = n2 * n;
        std::vector<cplx> tw(n / 2);
        for (int k = 0; k < n / 2; ++k) tw[k] = std::polar(1.0, -2.0 * M_PI * k / n);
        // 1 / lambda of the 7-point Laplacian per mode (h = 1); the mean mode is dropped
        std::vector<double> inv_k2(n3);
        std::vector<double> s2(n);
        for (int k = 0; k < n; ++k) {
            const double s = std::sin(M_PI * k / n);
            s2[k] = 4.0 * s * s;
        }
        for (int z = 0; z < n; ++z)
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x) {
                    const double l = s2[z] + s2[y] + s2[x];
                    inv_k2[(size_t)z * n2 + (size_t)y * n + x] = l > 0.0 ? 1.0 / l : 0.0;
                }
        std::vector<double> per((size_t)nplace * nrho);
        // at most 16 threads, and at most about 1 GiB of boxes (24 bytes per cell each)
        const unsigned hw = std::thread::hardware_concurrency();
        size_t nt = std::min<size_t>(16, hw ? hw : 1);
        nt = std::max<size_t>(1, std::min(nt, ((size_t)1 << 30) / (24 * n3)));
        const int nthreads = (int)nt;
        std::atomic<bool> failed{false};
        auto work = [&](int t) {
            try {
                for (int p = t; p < nplace; p += nthreads)
                    one_placement(n, nrho, drho, src + 3 * (size_t)p, dir + 3 * (size_t)p * nrho,
                                  tw, inv_k2, &per[(size_t)p * nrho]);
            } catch (...) {
                failed = true;
            }
        };
        std::vector<std::thread> pool;
        int started = 1;  // share 0 is the calling thread's
        try {
            for (int t = 1; t < nthreads; ++t) {
                pool.emplace_back(work, t);
                ++started;
            }
        } catch (...) {
        }
        work(0);
        for (int t = started; t < nthreads; ++t) work(t);  // shares whose thread did not start
        for (auto& th : pool) th.join();
        if (failed) return DISCOS_E_CAPACITY;
        // average in placement order, independent of the thread count
        for (int k = 0; k < nrho; ++k) {
            double acc = 0.0;
            for (int p = 0; p < nplace; ++p) acc += per[(size_t)p * nrho + k];
            g[k] = acc / nplace;
        }
        g[0] = 0.0;
    } catch (...) {
        return DISCOS_E_CAPACITY;
    }
    return DISCOS_OK;
}
