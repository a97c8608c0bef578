// Demagnetisation tensor of a regular grid and its Fourier spectrum (host, float64).
//
// The tensor N(r) between two cells offset by r is the cell average of the
// point-dipole kernel, N(r) = (1/V) int T(s) D(r+s) ds with the box
// autocorrelation T(s) = prod (h_d - |s_d|)_+ and D(p) = -(3 p p^T/|p|^2 - I)/(4 pi |p|^3);
// it discretises the paper's dipole-dipole field term (Methods).  Close cells
// use Newell, Williams & Dunlop's closed form (J. Geophys. Res. 98, 9551, 1993);
// separated cells use Gauss-Jacobi quadrature of the integral on each half of
// the tent (weight (h - s) on [0, h]), because the closed form cancels
// catastrophically (~eps R^6).
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

// Far field: the tent integral by Gauss-Jacobi quadrature.  On each half of
// the tent, int_0^h (h - s) f(s) ds = (h^2 / 4) int_{-1}^{1} (1 - x) f(h (1 + x) / 2) dx,
// a Jacobi weight (1 - x)^1 (1 + x)^0.  Its n-point Gauss rule (exact for
// polynomials of degree 2n - 1) has nodes at the eigenvalues of the Jacobi
// matrix of the monic recurrence, here diagonal a_k = -1 / ((2k + 1)(2k + 3))
// and off-diagonal b_k = sqrt(k (k + 1)) / (2k + 1); the nodes are found by
// Sturm-sequence bisection and the weights from the orthonormal polynomials,
// w_i = mu_0 / sum_k q_k(x_i)^2 with mu_0 = int (1 - x) dx = 2.
struct Rule1 {
    std::vector<double> s, w;  // nodes on [-h, h] and weights of int (h - |s|) f(s) ds
};

void jacobi10_rule(int n, std::vector<double>& x, std::vector<double>& w) {
    std::vector<double> a(n), b(n, 0.0);  // b[k] couples rows k-1 and k
    for (int k = 0; k < n; ++k) {
        a[k] = -1.0 / ((2.0 * k + 1.0) * (2.0 * k + 3.0));
        if (k > 0) b[k] = std::sqrt((double)k * (k + 1.0)) / (2.0 * k + 1.0);
    }
    // number of eigenvalues below t (Sturm sequence of the leading minors)
    auto below = [&](double t) {
        int cnt = 0;
        double d = 1.0;
        for (int k = 0; k < n; ++k) {
            d = (a[k] - t) - (k > 0 ? b[k] * b[k] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++cnt;
        }
        return cnt;
    };
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double lo = -1.0, hi = 1.0;  // every node lies inside (-1, 1)
        for (int it = 0; it < 200 && hi - lo > 4e-17; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (below(mid) > i) hi = mid; else lo = mid;
        }
        const double t = 0.5 * (lo + hi);
        // orthonormal polynomials q_k(t): q_0 = 1 / sqrt(mu_0) up to the common factor
        double q0 = 1.0, q1 = (t - a[0]) / (n > 1 ? b[1] : 1.0), sum = 1.0;
        if (n > 1) sum += q1 * q1;
        for (int k = 1; k + 1 < n; ++k) {
            const double q2 = ((t - a[k]) * q1 - b[k] * q0) / b[k + 1];
            sum += q2 * q2;
            q0 = q1;
            q1 = q2;
        }
        x[i] = t;
        w[i] = 2.0 / sum;
    }
}

// Both halves of the tent on [-h, h], n nodes each.
void tent_jacobi(double h, int n, Rule1& r) {
    std::vector<double> x, w;
    jacobi10_rule(n, x, w);
    r.s.assign(2 * n, 0.0);
    r.w.assign(2 * n, 0.0);
    for (int i = 0; i < n; ++i) {
        const double si = 0.5 * h * (1.0 + x[i]);
        const double wi = 0.25 * h * h * w[i];
        r.s[i] = si;
        r.w[i] = wi;
        r.s[n + i] = -si;
        r.w[n + i] = wi;
    }
}

struct Rule3 {
    Rule1 x, y, z;
};

// N(r) = (1/V) sum_ijk W_i W_j W_k D(r + (s_i, s_j, s_k)), D(p) = (I/|p|^3 - 3 p p^T/|p|^5) / (4 pi).
void tent_sum(double X, double Y, double Z, double V, const Rule3& q, double o[6]) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (size_t k = 0; k < q.z.s.size(); ++k) {
        const double pz = Z + q.z.s[k];
        for (size_t j = 0; j < q.y.s.size(); ++j) {
            const double py = Y + q.y.s[j];
            const double wjk = q.y.w[j] * q.z.w[k];
            for (size_t i = 0; i < q.x.s.size(); ++i) {
                const double px = X + q.x.s[i];
                const double p2 = px * px + py * py + pz * pz;
                const double inv = 1.0 / (p2 * std::sqrt(p2));  // |p|^-3
                const double w = wjk * q.x.w[i] * inv;
                const double w3 = 3.0 * w / p2;                  // 3 w |p|^-2
                acc[0] += w - w3 * px * px;
                acc[1] += w - w3 * py * py;
                acc[2] += w - w3 * pz * pz;
                acc[3] -= w3 * px * py;
                acc[4] -= w3 * px * pz;
                acc[5] -= w3 * py * pz;
            }
        }
    }
    const double c = 1.0 / (4.0 * kPi * V);
    for (int i = 0; i < 6; ++i) o[i] = acc[i] * c;
}

const Rule3& rule3(double hx, double hy, double hz, int n) {
    // per-thread cache keyed on the cell and the order; a problem uses one cell shape
    struct Entry {
        double hx, hy, hz;
        int n;
        Rule3 r;
    };
    static thread_local std::vector<Entry> cache;
    for (auto& e : cache)
        if (e.hx == hx && e.hy == hy && e.hz == hz && e.n == n) return e.r;
    Entry e{hx, hy, hz, n, {}};
    tent_jacobi(hx, n, e.r.x);
    tent_jacobi(hy, n, e.r.y);
    tent_jacobi(hz, n, e.r.z);
    cache.push_back(std::move(e));
    return cache.back().r;
}

// Nodes per tent half for centres q = |r| / h_max apart (q >= 2).  The
// integrand's singularity at r + s = 0 moves away from the integration box as q
// grows, so Gauss convergence is geometric in q; the orders keep the rule's
// error near 1e-14 of the largest component (checked against the closed form
// and against 96-point Gauss-Legendre quadrature of the same integral).
int far_order(double q) {
    return q < 2.0 ? 20 : (q < 3.0 ? 16 : (q < 5.0 ? 12 : (q < 10.0 ? 8 : (q < 24.0 ? 6 : (q < 64.0 ? 4 : 3)))));
}

}  // namespace

void tensor_at_mode(double X, double Y, double Z, double hx, double hy, double hz, int mode, double out[6]) {
    // mode 0: closed form for centres less than two largest cell edges apart,
    // the tent quadrature beyond (there it is accurate to ~1e-14 while the
    // closed form's cancellation grows like the sixth power of the distance);
    // 1: closed form only; 2: quadrature only.
    const double hm = std::fmax(hx, std::fmax(hy, hz));
    const double q = std::sqrt(X * X + Y * Y + Z * Z) / hm;
    const bool closed = mode == 1 || (mode == 0 && q < 2.0);
    if (closed) {
        closed_form(X, Y, Z, hx, hy, hz, out);
        return;
    }
    tent_sum(X, Y, Z, hx * hy * hz, rule3(hx, hy, hz, far_order(q)), out);
}

void tensor_at(double X, double Y, double Z, double hx, double hy, double hz, double out[6]) {
    tensor_at_mode(X, Y, Z, hx, hy, hz, 0, out);
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
