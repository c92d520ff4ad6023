// Host thermodynamics: Eq. (17) (Carnahan-Starling hard spheres plus a mean-field
// attraction) and the van der Waals form; coexistence by the equal chemical
// potential / equal pressure conditions.
#include "thermo.hpp"

#include <cmath>

namespace lbm_host {

namespace {
// Critical-point coefficients of the Carnahan-Starling form, Eq. (17):
// a~ = 0.4963880577294099 R^2 Tc^2 / pc and b~ = 0.1872945669467330 R Tc / pc.
constexpr long double kCsA = 0.4963880577294099L;
constexpr long double kCsB = 0.1872945669467330L;
}  // namespace

long double density_limit(const Eos& e) {
    return e.kind == 0 ? 4.0L / e.b : 1.0L / e.b;
}

long double pressure(const Eos& e, long double rho, long double T) {
    if (e.kind == 0) {
        const long double t = 0.25L * e.b * rho, s = 1.0L - t;
        const long double z = (1.0L + t * (1.0L + t * (1.0L - t))) / (s * s * s);
        return e.K * (rho * e.R * T * z - e.a * rho * rho);
    }
    return e.K * (rho * e.R * T / (1.0L - e.b * rho) - e.a * rho * rho);
}

long double pressure_slope(const Eos& e, long double rho, long double T) {
    if (e.kind == 0) {
        // d(rho Z)/d rho = (1 + 4t + 4t^2 - 4t^3 + t^4) / (1 - t)^4
        const long double t = 0.25L * e.b * rho, s = 1.0L - t;
        const long double num = 1.0L + t * (4.0L + t * (4.0L + t * (-4.0L + t)));
        return e.K * (e.R * T * num / (s * s * s * s) - 2.0L * e.a * rho);
    }
    const long double s = 1.0L - e.b * rho;
    return e.K * (e.R * T / (s * s) - 2.0L * e.a * rho);
}

long double chem_potential(const Eos& e, long double rho, long double T) {
    if (e.kind == 0) {
        // hard-sphere excess part (8t - 9t^2 + 3t^3) / (1 - t)^3
        const long double t = 0.25L * e.b * rho, s = 1.0L - t;
        const long double ex = t * (8.0L + t * (-9.0L + 3.0L * t)) / (s * s * s);
        return e.K * (e.R * T * (std::log(rho) + ex) - 2.0L * e.a * rho);
    }
    const long double s = 1.0L - e.b * rho;
    return e.K * (e.R * T * (std::log(rho / s) + e.b * rho / s) - 2.0L * e.a * rho);
}

void critical(const Eos& e, long double* Tc, long double* pc) {
    if (e.kind == 0) {
        *Tc = (e.a / e.b) * (kCsB / kCsA) / e.R;
        *pc = e.K * kCsB * e.R * (*Tc) / e.b;
    } else {
        *Tc = 8.0L * e.a / (27.0L * e.b * e.R);
        *pc = e.K * e.a / (27.0L * e.b * e.b);
    }
}

namespace {

// Root of g on [lo, hi] where g(lo) and g(hi) differ in sign; plain bisection to
// the last bit of long double.
template <class F>
long double bisect(F g, long double lo, long double hi) {
    long double glo = g(lo);
    for (int it = 0; it < 200; ++it) {
        const long double mid = 0.5L * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const long double gm = g(mid);
        if ((gm > 0) == (glo > 0)) { lo = mid; glo = gm; } else { hi = mid; }
    }
    return 0.5L * (lo + hi);
}

}  // namespace

bool coexistence(const Eos& e, long double T, long double* rho_v, long double* rho_l,
                 long double* p_s, std::string* err) {
    const long double rmax = density_limit(e);
    // 1. spinodals: the two zeros of dp/drho, by a sign scan then bisection
    long double sp[2];
    int nsp = 0;
    const int nscan = 20000;
    long double prev_r = 0, prev_v = 0;
    for (int k = 1; k < nscan && nsp < 2; ++k) {
        const long double r = rmax * k / nscan;
        const long double v = pressure_slope(e, r, T);
        if (k > 1 && ((v > 0) != (prev_v > 0)))
            sp[nsp++] = bisect([&](long double x) { return pressure_slope(e, x, T); }, prev_r, r);
        prev_r = r;
        prev_v = v;
    }
    if (nsp != 2) {
        if (err) *err = "temperature is not below the critical temperature of the EOS";
        return false;
    }
    // 2. for a trial saturation pressure, the vapour root lies below the first
    //    spinodal and the liquid root above the second; bisect mu_l - mu_v in p
    auto vap = [&](long double ps) {
        return bisect([&](long double x) { return pressure(e, x, T) - ps; }, 1e-30L, sp[0]);
    };
    auto liq = [&](long double ps) {
        long double hi = sp[1] + 0.5L * (rmax - sp[1]);
        while (pressure(e, hi, T) < ps) hi += 0.5L * (rmax - hi);
        return bisect([&](long double x) { return pressure(e, x, T) - ps; }, sp[1], hi);
    };
    auto dmu = [&](long double ps) {
        return chem_potential(e, liq(ps), T) - chem_potential(e, vap(ps), T);
    };
    long double plo = pressure(e, sp[1], T);
    if (plo < 0) plo = 0;
    plo += 1e-30L;
    long double phi = pressure(e, sp[0], T) * (1.0L - 1e-15L);
    if ((dmu(plo) > 0) == (dmu(phi) > 0)) {
        if (err) *err = "could not bracket the coexistence pressure";
        return false;
    }
    const long double ps = bisect(dmu, plo, phi);
    long double rv = vap(ps), rl = liq(ps);
    // 3. Newton on (rho_v, rho_l): p_v - p_l = 0, mu_v - mu_l = 0, using dmu/drho = p'/rho
    for (int it = 0; it < 30; ++it) {
        const long double f1 = pressure(e, rv, T) - pressure(e, rl, T);
        const long double f2 = chem_potential(e, rv, T) - chem_potential(e, rl, T);
        const long double pv = pressure_slope(e, rv, T), pl = pressure_slope(e, rl, T);
        const long double a11 = pv, a12 = -pl, a21 = pv / rv, a22 = -pl / rl;
        const long double det = a11 * a22 - a12 * a21;
        if (det == 0) break;
        const long double dv = (f1 * a22 - a12 * f2) / det;
        const long double dl = (a11 * f2 - a21 * f1) / det;
        rv -= dv;
        rl -= dl;
        if (std::fabs(dv) <= 1e-19L * rv && std::fabs(dl) <= 1e-19L * rl) break;
    }
    if (!(rv > 0 && rv < rl && rl < rmax)) {
        if (err) *err = "coexistence iteration left the admissible density range";
        return false;
    }
    *rho_v = rv;
    *rho_l = rl;
    *p_s = pressure(e, rv, T);
    return true;
}

namespace {

// Composite 20-point Gauss-Legendre rule on `panels` equal panels of [a, b].
template <class F>
long double gauss_legendre(F f, long double a, long double b, int panels) {
    // nodes and weights of the 20-point rule on [-1, 1] (positive half; symmetric)
    static const long double x[10] = {
        0.0765265211334973337546404093988382L, 0.2277858511416450780804961953685746L,
        0.3737060887154195606725481770249272L, 0.5108670019508270980043640509552510L,
        0.6360536807265150254528366962262859L, 0.7463319064601507926143050703556416L,
        0.8391169718222188233945290617015207L, 0.9122344282513259058677524412032981L,
        0.9639719272779137912676661311972772L, 0.9931285991850949247861223884713203L};
    static const long double w[10] = {
        0.1527533871307258506980843319550976L, 0.1491729864726037467878287370019694L,
        0.1420961093183820513292983250671649L, 0.1316886384491766268984944997481631L,
        0.1181945319615184173123773777113823L, 0.1019301198172404350367501354803499L,
        0.0832767415767047487247581432220463L, 0.0626720483341090635695065351870416L,
        0.0406014298003869413310399522749321L, 0.0176140071391521183118619623518528L};
    const long double h = (b - a) / panels;
    long double sum = 0;
    for (int k = 0; k < panels; ++k) {
        const long double mid = a + (k + 0.5L) * h, half = 0.5L * h;
        long double ps = 0;
        for (int j = 0; j < 10; ++j) ps += w[j] * (f(mid - half * x[j]) + f(mid + half * x[j]));
        sum += half * ps;
    }
    return sum;
}

}  // namespace

bool interface_sigma_width(const Eos& e, long double T, long double kappa, long double* sigma, long double* W,
                           std::string* err) {
    long double rv, rl, ps;
    if (!coexistence(e, T, &rv, &rl, &ps, err)) return false;
    const long double mus = chem_potential(e, rv, T);
    // grand-potential excess over the tie line: rho (mu - mu_s) - (p - p_s) >= 0
    auto dom = [&](long double r) {
        const long double v = r * (chem_potential(e, r, T) - mus) - (pressure(e, r, T) - ps);
        return v > 0 ? v : 0.0L;
    };
    *sigma = gauss_legendre([&](long double r) { return std::sqrt(2.0L * kappa * dom(r)); }, rv, rl, 256);
    const long double r5 = rv + 0.05L * (rl - rv), r95 = rv + 0.95L * (rl - rv);
    *W = gauss_legendre([&](long double r) { return std::sqrt(kappa / (2.0L * dom(r))); }, r5, r95, 256);
    if (!(std::isfinite(*sigma) && std::isfinite(*W) && *sigma > 0 && *W > 0)) {
        if (err) *err = "interface integrals did not converge";
        return false;
    }
    return true;
}

bool vapour_root(const Eos& e, long double T, long double p, long double* rho, std::string* err) {
    // the first zero of dp/drho bounds the vapour branch, on which p rises with rho
    const long double rmax = density_limit(e);
    const int nscan = 20000;
    long double top = -1, prev_r = 0, prev_v = 0;
    for (int k = 1; k < nscan; ++k) {
        const long double r = rmax * k / nscan;
        const long double v = pressure_slope(e, r, T);
        if (k > 1 && ((v > 0) != (prev_v > 0))) {
            top = bisect([&](long double x) { return pressure_slope(e, x, T); }, prev_r, r);
            break;
        }
        prev_r = r;
        prev_v = v;
    }
    if (top < 0) top = rmax * (1.0L - 1e-12L);  // supercritical: p rises everywhere
    if (!(p > 0) || !(pressure(e, top, T) > p)) {
        if (err) *err = "the pressure is not reached on the vapour branch at this temperature";
        return false;
    }
    *rho = bisect([&](long double x) { return pressure(e, x, T) - p; }, 1e-30L, top);
    return true;
}

}  // namespace lbm_host
