// Host thermodynamics of the library: equation of state, Maxwell coexistence
// and the per-run constants of the model.  Long double throughout; results are
// rounded to double once.
#pragma once

#include <string>

namespace lbm_host {

struct Eos {
    int kind;          // 0 = Carnahan-Starling with attraction (Eq. (17)), 1 = van der Waals
    long double a, b, R, K;
};

// Pressure p_EOS(rho, T) and its rho-derivative at fixed T.
long double pressure(const Eos& e, long double rho, long double T);
long double pressure_slope(const Eos& e, long double rho, long double T);
// Chemical potential up to a function of T only.
long double chem_potential(const Eos& e, long double rho, long double T);
// Largest admissible density (packing fraction 1).
long double density_limit(const Eos& e);
// Critical temperature and pressure.
void critical(const Eos& e, long double* Tc, long double* pc);
// Coexisting densities and pressure at T < Tc.  Returns false (with a message) on failure.
bool coexistence(const Eos& e, long double T, long double* rho_v, long double* rho_l,
                 long double* p_s, std::string* err);
// Density on the vapour branch (below the first spinodal) at which p_EOS(rho, T) = p.
// Returns false (with a message) when p is not reached there.
bool vapour_root(const Eos& e, long double T, long double p, long double* rho, std::string* err);
// Square-gradient surface tension sigma = int sqrt(2 kappa dOmega) drho over [rho_v, rho_l]
// and 5 %-95 % width W = int sqrt(kappa / (2 dOmega)) drho of the flat interface at T,
// with dOmega the grand-potential excess over the coexistence tie line.
bool interface_sigma_width(const Eos& e, long double T, long double kappa, long double* sigma, long double* W,
                           std::string* err);

}  // namespace lbm_host
