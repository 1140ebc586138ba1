// lbm_eos_host.hpp -- host-side Peng-Robinson quantities the step needs:
// critical point (Tc, rho_c are not printed in the paper, Sec 2.2), alpha(T),
// and the Maxwell coexistence densities used to set up initial states.
#pragma once

#include <cmath>

namespace lbm {

struct PR {
    double a, b, R, omega;
};

inline double pr_pressure(const PR& e, double aa, double T, double rho)
{
    const double x = e.b * rho;
    return rho * e.R * T / (1.0 - x) - aa * rho * rho / (1.0 + 2.0 * x - x * x);
}

// d p / d rho of Eq 14 at fixed T.
inline double pr_dpdrho(const PR& e, double aa, double T, double rho)
{
    const double x = e.b * rho, g = 1.0 - x, D = 1.0 + 2.0 * x - x * x;
    return e.R * T / (g * g) - aa * 2.0 * rho * (1.0 + x) / (D * D);
}

// psi'(rho) of Eq 15 (no gradient term), written out term by term.
inline double pr_mu(const PR& e, double aa, double T, double rho)
{
    const double s2 = std::sqrt(2.0), x = e.b * rho;
    return e.R * T * std::log(rho / (1.0 - x)) - aa / (2.0 * s2 * e.b) * std::log((s2 - 1.0 + x) / (s2 + 1.0 - x))
         + e.R * T / (1.0 - x) - aa * rho / (1.0 + 2.0 * x - x * x);
}

inline double pr_alpha(double Tr, double omega)
{
    const double m = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    const double s = 1.0 + m * (1.0 - std::sqrt(Tr));
    return s * s;
}

// Critical point with alpha = 1.  dp/drho = 0 gives R T(rho) in closed form;
// the critical density is the root of d2p/drho2 evaluated on that curve, found
// by bisection in x = b rho on (0, 1).
inline void pr_critical(const PR& e, double& Tc, double& rhoc, double& pc)
{
    auto RT_of = [&](double x) {   // from dp/drho = 0 with aa = a
        const double g = 1.0 - x, D = 1.0 + 2.0 * x - x * x;
        return e.a / e.b * 2.0 * x * (1.0 + x) * g * g / (D * D);
    };
    auto second = [&](double x) {  // b^-1 d2p/drho2 along the curve
        const double g = 1.0 - x, D = 1.0 + 2.0 * x - x * x;
        const double RT = RT_of(x);
        // d/drho [ R T rho / (1 - b rho) ] second derivative: 2 b R T / g^3
        const double ideal = 2.0 * RT / (g * g * g);
        // d2/drho2 [ a rho^2 / D ] / b: derivative of 2 a rho (1+x)/D^2 w.r.t rho, over b
        // = (a/b) [2 (1 + 2x) D - 8 x (1 + x)(1 - x)] / D^3
        const double attr = e.a / e.b * (2.0 * (1.0 + 2.0 * x) * D - 8.0 * x * (1.0 + x) * (1.0 - x)) / (D * D * D);
        return ideal - attr;
    };
    double lo = 1e-6, hi = 0.9;
    double slo = second(lo);
    for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (lo + hi);
        const double sm = second(m);
        if ((sm > 0.0) == (slo > 0.0)) { lo = m; slo = sm; } else { hi = m; }
    }
    const double x = 0.5 * (lo + hi);
    rhoc = x / e.b;
    Tc = RT_of(x) / e.R;
    pc = pr_pressure(e, e.a, Tc, rhoc);
}

// Maxwell construction: the saturation pressure P at which the gas and liquid
// roots of p(rho) = P have equal chemical potential.  Roots by bisection on the
// monotone branches outside the spinodal interval; P by bisection in log P.
inline bool pr_coexistence(const PR& e, double Tr, double& rho_g, double& rho_l)
{
    if (!(Tr > 0.0 && Tr < 1.0)) return false;
    double Tc, rc, pc;
    pr_critical(e, Tc, rc, pc);
    const double T = Tr * Tc, aa = e.a * pr_alpha(Tr, e.omega);
    const double top = (1.0 / e.b) * (1.0 - 1e-14);
    // spinodal interval: dp/drho < 0 between the two roots around the
    // inflection near rho_c
    double s_lo = rc, s_hi = rc;
    if (pr_dpdrho(e, aa, T, rc) >= 0.0) return false;
    {
        double lo = 0.0, hi = rc;
        for (int it = 0; it < 300; ++it) {
            const double m = 0.5 * (lo + hi);
            if (pr_dpdrho(e, aa, T, m) > 0.0) lo = m; else hi = m;
        }
        s_lo = lo;
        lo = rc; hi = top;
        for (int it = 0; it < 300; ++it) {
            const double m = 0.5 * (lo + hi);
            if (pr_dpdrho(e, aa, T, m) < 0.0) lo = m; else hi = m;
        }
        s_hi = hi;
    }
    auto root = [&](double P, double lo, double hi) {
        // p increasing on [lo, hi]; geometric bisection when the bracket is wide
        for (int it = 0; it < 3000 && hi - lo > 4e-16 * hi; ++it) {
            const double m = (lo > 0.0 && hi > 8.0 * lo) ? std::sqrt(lo * hi) : 0.5 * (lo + hi);
            if (pr_pressure(e, aa, T, m) < P) lo = m; else hi = m;
        }
        return 0.5 * (lo + hi);
    };
    double Phi = pr_pressure(e, aa, T, s_lo);
    double Plo = std::max(pr_pressure(e, aa, T, s_hi), 1e-300);
    double g = 0.0, l = 0.0;
    for (int it = 0; it < 400; ++it) {
        const double P = std::sqrt(Plo * Phi);
        g = root(P, 0.0, s_lo);
        l = root(P, s_hi, top);
        const double d = pr_mu(e, aa, T, l) - pr_mu(e, aa, T, g);
        if (d > 0.0) Plo = P; else Phi = P;
        if (Phi - Plo <= 2e-16 * Phi) break;
    }
    rho_g = g;
    rho_l = l;
    return true;
}

}  // namespace lbm
