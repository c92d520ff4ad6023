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

}  // namespace lbm_host
