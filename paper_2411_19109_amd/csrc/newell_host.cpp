// Demagnetisation tensor of a regular grid and its Fourier spectrum (host, float64).
//
// The tensor N(r) between two cells offset by r is the cell average of the
// point-dipole kernel, N(r) = (1/V) int T(s) D(r+s) ds with the box
// autocorrelation T(s) = prod (h_d - |s_d|)_+ and D(p) = -(3 p p^T/|p|^2 - I)/(4 pi |p|^3);
// it discretises the paper's dipole-dipole field term (Methods).  Close cells
// use Newell, Williams & Dunlop's closed form (J. Geophys. Res. 98, 9551, 1993);
// separated cells use Gauss-Legendre quadrature of the integral, split at the
// tent's kink, because the closed form cancels catastrophically (~eps R^6).
//
// The spectrum is the DFT of the zero-padded kernel.  The diagonal components
// are even in every offset and the off-diagonal ones odd in their two axes, so
// each spectrum is real and follows from separable cosine / sine sums over the
// non-negative octant of offsets; only ky <= Py/2, kz <= Pz/2 are stored.
#include <cmath>
#include <thread>
#include <vector>

#include "llg_internal.hpp"

namespace llg {
namespace {

constexpr double kPi = 3.14159265358979323846;

double asinh_ratio(double num, double den2) { return den2 > 0.0 ? std::asinh(num / std::sqrt(den2)) : 0.0; }
double atan_ratio(double num, double den) { return den != 0.0 ? std::atan(num / den) : 0.0; }

double newell_f(double x, double y, double z) {
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = std::sqrt(x2 + y2 + z2);
    double r = (2.0 * x2 - y2 - z2) * R / 6.0;
    r += 0.5 * y * (z2 - x2) * asinh_ratio(y, x2 + z2);
    r += 0.5 * z * (y2 - x2) * asinh_ratio(z, x2 + y2);
    r -= x * y * z * atan_ratio(y * z, x * R);
    return r;
}

double newell_g(double x, double y, double z) {
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = std::sqrt(x2 + y2 + z2);
    double r = -x * y * R / 3.0;
    r += x * y * z * asinh_ratio(z, x2 + y2);
    r += y * (3.0 * z2 - y2) * asinh_ratio(x, y2 + z2) / 6.0;
    r += x * (3.0 * z2 - x2) * asinh_ratio(y, x2 + z2) / 6.0;
    r -= z * z2 * atan_ratio(x * y, z * R) / 6.0;
    r -= 0.5 * z * y2 * atan_ratio(x * z, y * R);
    r -= 0.5 * z * x2 * atan_ratio(y * z, x * R);
    return r;
}

template <typename F>
double second_diff(F fn, double X, double Y, double Z, double a, double b, double c) {
    static const double w[3] = {-1.0, 2.0, -1.0};
    double acc = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                acc += w[i] * w[j] * w[k] * fn(X + (i - 1) * a, Y + (j - 1) * b, Z + (k - 1) * c);
    return acc;
}

void closed_form(double X, double Y, double Z, double hx, double hy, double hz, double o[6]) {
    const double c = 1.0 / (4.0 * kPi * hx * hy * hz);
    o[0] = c * second_diff(newell_f, X, Y, Z, hx, hy, hz);
    o[1] = c * second_diff(newell_f, Y, X, Z, hy, hx, hz);
    o[2] = c * second_diff(newell_f, Z, Y, X, hz, hy, hx);
    o[3] = c * second_diff(newell_g, X, Y, Z, hx, hy, hz);
    o[4] = c * second_diff(newell_g, X, Z, Y, hx, hz, hy);
    o[5] = c * second_diff(newell_g, Y, Z, X, hy, hz, hx);
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double t = std::cos(kPi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(t), p0 = P_{n-1}(t)
            double dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

// Nodes s and weights on [-h, h] for int (h - |s|) f(s) ds, n points per half.
void tent_rule(double h, int n, std::vector<double>& s, std::vector<double>& ws) {
    std::vector<double> t, w;
    gauss_legendre(n, t, w);
    s.resize(2 * n);
    ws.resize(2 * n);
    for (int i = 0; i < n; ++i) {
        double si = 0.5 * h * (t[i] + 1.0);
        double wi = 0.5 * h * w[i] * (h - si);
        s[i] = si;
        ws[i] = wi;
        s[n + i] = -si;
        ws[n + i] = wi;
    }
}

struct Rule {
    std::vector<double> sx, wx, sy, wy, sz, wz;
};

void quadrature(double X, double Y, double Z, double V, const Rule& q, double o[6]) {
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (size_t i = 0; i < q.sx.size(); ++i) {
        const double px = X + q.sx[i];
        for (size_t j = 0; j < q.sy.size(); ++j) {
            const double py = Y + q.sy[j];
            const double wij = q.wx[i] * q.wy[j];
            for (size_t k = 0; k < q.sz.size(); ++k) {
                const double pz = Z + q.sz[k];
                const double r2 = px * px + py * py + pz * pz;
                const double ir = 1.0 / std::sqrt(r2);
                const double ir3 = ir / r2, ir5 = ir3 / r2;
                const double w = wij * q.wz[k];
                a[0] += w * (ir3 - 3.0 * px * px * ir5);
                a[1] += w * (ir3 - 3.0 * py * py * ir5);
                a[2] += w * (ir3 - 3.0 * pz * pz * ir5);
                a[3] += w * (-3.0 * px * py * ir5);
                a[4] += w * (-3.0 * px * pz * ir5);
                a[5] += w * (-3.0 * py * pz * ir5);
            }
        }
    }
    const double c = 1.0 / (4.0 * kPi * V);
    for (int i = 0; i < 6; ++i) o[i] = a[i] * c;
}

const Rule& rule_for(double hx, double hy, double hz, int n) {
    // small cache keyed on (h, n); problems use a single cell shape
    struct Entry { double hx, hy, hz; int n; Rule r; };
    static thread_local std::vector<Entry> cache;
    for (auto& e : cache)
        if (e.hx == hx && e.hy == hy && e.hz == hz && e.n == n) return e.r;
    Entry e{hx, hy, hz, n, {}};
    tent_rule(hx, n, e.r.sx, e.r.wx);
    tent_rule(hy, n, e.r.sy, e.r.wy);
    tent_rule(hz, n, e.r.sz, e.r.wz);
    cache.push_back(std::move(e));
    return cache.back().r;
}

}  // namespace

void tensor_at(double X, double Y, double Z, double hx, double hy, double hz, double out[6]) {
    // Euclidean distance of the nearest point of the integrand's support from
    // the origin, in units of the largest edge: closed form below 1.5,
    // quadrature above (8 / 5 / 4 points per half-axis as the gap grows).
    const double gx = std::fmax(std::fabs(X) - hx, 0.0);
    const double gy = std::fmax(std::fabs(Y) - hy, 0.0);
    const double gz = std::fmax(std::fabs(Z) - hz, 0.0);
    const double q = std::sqrt(gx * gx + gy * gy + gz * gz) / std::fmax(hx, std::fmax(hy, hz));
    if (q < 1.5) {
        closed_form(X, Y, Z, hx, hy, hz, out);
        return;
    }
    const int n = q <= 8.0 ? 8 : (q <= 30.0 ? 5 : 4);
    quadrature(X, Y, Z, hx * hy * hz, rule_for(hx, hy, hz, n), out);
}

void build_tensor_spectrum(int nx, int ny, int nz, double dx, double dy, double dz, int Px, int Py, int Pz,
                           double scale, std::vector<double>& out, int& ncomp) {
    const size_t Noct = (size_t)nx * ny * nz;
    std::vector<double> oct(6 * Noct);
    // tensor over the non-negative octant of offsets, in parallel over rows
    unsigned nth = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    const int rows = ny * nz;
    for (unsigned t = 0; t < nth; ++t) {
        pool.emplace_back([&, t]() {
            for (int r = (int)t; r < rows; r += (int)nth) {
                const int j = r % ny, k = r / ny;
                for (int i = 0; i < nx; ++i) {
                    double o[6];
                    tensor_at(i * dx, j * dy, k * dz, dx, dy, dz, o);
                    const size_t idx = (size_t)i + (size_t)nx * r;
                    for (int c = 0; c < 6; ++c) oct[c * Noct + idx] = o[c];
                }
            }
        });
    }
    for (auto& th : pool) th.join();

    ncomp = nz > 1 ? 6 : 4;
    const int Kx = Px / 2 + 1, Ky = Py / 2 + 1, Kz = Pz / 2 + 1;
    // per-axis real transforms of an even (E) or odd (O) sequence of offsets 0..n-1:
    //   E[k] = sum_X w_X a_X cos(2 pi k X / P), w_0 = 1, w_X = 2
    //   O[k] = -2 sum_{X>=1} a_X sin(2 pi k X / P)        (the factor i is applied below)
    auto table = [](int n, int P, int K, bool odd) {
        std::vector<double> t((size_t)K * n);
        for (int k = 0; k < K; ++k)
            for (int X = 0; X < n; ++X) {
                const double th = 2.0 * kPi * (double)(((long long)k * X) % P) / P;
                t[(size_t)k * n + X] = odd ? (X == 0 ? 0.0 : -2.0 * std::sin(th)) : (X == 0 ? 1.0 : 2.0) * std::cos(th);
            }
        return t;
    };
    const auto Ex = table(nx, Px, Kx, false), Ox = table(nx, Px, Kx, true);
    const auto Ey = table(ny, Py, Ky, false), Oy = table(ny, Py, Ky, true);
    const auto Ez = table(nz, Pz, Kz, false), Oz = table(nz, Pz, Kz, true);
    // component c: parity flags (odd in x, odd in y, odd in z) and sign (i^2 = -1 for two odd axes)
    const int oddx[6] = {0, 0, 0, 1, 1, 0}, oddy[6] = {0, 0, 0, 1, 0, 1}, oddz[6] = {0, 0, 0, 0, 1, 1};
    const double sgn[6] = {1, 1, 1, -1, -1, -1};
    out.assign((size_t)ncomp * Kz * Ky * Kx, 0.0);
    for (int c = 0; c < ncomp; ++c) {
        const auto& TX = oddx[c] ? Ox : Ex;
        const auto& TY = oddy[c] ? Oy : Ey;
        const auto& TZ = oddz[c] ? Oz : Ez;
        const double* a = &oct[(size_t)c * Noct];
        // x transform: rows (z, y) -> (z, y, kx)
        std::vector<double> t1((size_t)nz * ny * Kx);
        for (int r = 0; r < ny * nz; ++r)
            for (int k = 0; k < Kx; ++k) {
                double s = 0.0;
                for (int X = 0; X < nx; ++X) s += TX[(size_t)k * nx + X] * a[(size_t)r * nx + X];
                t1[(size_t)r * Kx + k] = s;
            }
        // y transform: (z, y, kx) -> (z, ky, kx)
        std::vector<double> t2((size_t)nz * Ky * Kx);
        for (int z = 0; z < nz; ++z)
            for (int ky = 0; ky < Ky; ++ky)
                for (int k = 0; k < Kx; ++k) {
                    double s = 0.0;
                    for (int Y = 0; Y < ny; ++Y) s += TY[(size_t)ky * ny + Y] * t1[((size_t)z * ny + Y) * Kx + k];
                    t2[((size_t)z * Ky + ky) * Kx + k] = s;
                }
        // z transform: (z, ky, kx) -> (kz, ky, kx)
        for (int kz = 0; kz < Kz; ++kz)
            for (int ky = 0; ky < Ky; ++ky)
                for (int k = 0; k < Kx; ++k) {
                    double s = 0.0;
                    for (int Z = 0; Z < nz; ++Z) s += TZ[(size_t)kz * nz + Z] * t2[((size_t)Z * Ky + ky) * Kx + k];
                    out[(((size_t)c * Kz + kz) * Ky + ky) * Kx + k] = sgn[c] * s * scale;
                }
    }
}

}  // namespace llg
