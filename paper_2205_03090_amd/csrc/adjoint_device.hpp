// adjoint_device.hpp -- vector-Jacobian product of the converged split by the
// implicit function theorem, one mixture per lane.
//
// The split n^V = u solves r(u; p) = ln y + ln phi(y) - ln x - ln phi(x) = 0
// (the equilibrium condition eq_cond in logarithms; eq. split_grad) with
// z~ = z/sum z, x = (z~ - u)/(1 - beta), y = u/beta, beta = sum u.  The
// outputs o = (beta, x, y).  With H~ = dr/du (eq. split_hess, whose Cholesky
// factor the forward keeps) and cotangents o_bar:
//   u_bar = (do/du)^T o_bar,   H~ lambda = u_bar,
//   p_bar = (do/dp)^T o_bar - (dr/dp)^T lambda.
// The paper applies the same theorem to the Rachford-Rice root when training
// its initializer (Sec. 4.2.2); here it is applied to the whole split.
#pragma once

#include "srk_device.hpp"

namespace ptf {

// Contractions of lambda with the parameter derivatives of ln phi of one
// phase at composition c (normalised): d(lambda . ln phi)/dT, /dP and, for
// each pair a < b, the derivative for a symmetric perturbation of k_ab = k_ba.
// With Lb = sum lambda_i B_i, L1 = sum lambda_i, Lp = sum lambda_i psi_i
// (psi_i = s_i psi'_i), lambda . ln phi = Lb q1 - L1 ln(Z - B) - q2 Lp, and
// every quantity depends on the parameters through A, B, psi_i, B_i and Z(A, B)
// (implicit differentiation of the cubic: f_A = Z - B, f_B = -(1+2B)Z - A,
// f_Z = 3Z^2 - 2Z + A - B - B^2).
//   P: A, B, psi_i, B_i are all proportional to P.
//   T: s_i = |a_i| (Tc_i/T) sqrt(OMEGA_A P/Pc_i), a_i = 1 + m_i (1 - sqrt(T/Tc_i)),
//      so d ln s_i/dT = a_i'/a_i - 1/T = d_i; B_i ~ 1/T;
//      dA/dT = 2 sum_i c_i d_i psi_i, d psi_i/dT = s_i (d_i psi'_i + chi_i),
//      chi_i = sum_j (1 - k_ij) s_j c_j d_j.
//   k_ab: dA = -2 c_a c_b s_a s_b dk, d psi_a = -s_a s_b c_b dk, d psi_b = -s_a s_b c_a dk.
template <int NC>
struct PhaseGrad {
    double dT, dP;
    double dk[NC * (NC - 1) / 2];   // pairs (a < b), row-major over a
};

template <int NC>
__device__ __forceinline__ void phase_param_vjp(PhaseGrad<NC> &out, const Phase<NC> &o,
                                                const Eos<NC> &e, const double (&c)[NC],
                                                const double (&lam)[NC],
                                                const double *__restrict__ K,
                                                const double *__restrict__ Tc,
                                                const double *__restrict__ om, double T,
                                                double P)
{
    const double A = o.A, B = o.B, Z = o.Z, L = o.L;
    const double ib = 1.0 / B;
    const double fA = Z - B;
    const double fB = -(1.0 + 2.0 * B) * Z - A;
    const double ifZ = 1.0 / ((3.0 * Z - 2.0) * Z + A - B - B * B);
    const double izzb = 1.0 / (Z * (Z + B));
    const double izb = 1.0 / (Z - B);
    double Lb = 0.0, L1 = 0.0, Lp = 0.0;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        Lb += lam[i] * e.b[i];
        L1 += lam[i];
        Lp += lam[i] * e.s[i] * o.psi[i];
    }
    // generic first-order change of lambda . ln phi for changes dA, dB (with
    // B_i and psi_i changes handled by the callers)
    auto core = [&](double dA, double dB) {
        const double dZ = -(fA * dA + fB * dB) * ifZ;
        const double dL = (Z * dB - B * dZ) * izzb;
        const double dlzb = (dZ - dB) * izb;
        const double dq1 = (dZ + (dA * L + A * dL) * ib - A * L * dB * ib * ib) * ib - o.q1 * dB * ib;
        const double dq2 = 2.0 * (dL - L * dB * ib) * ib;
        return Lb * dq1 - L1 * dlzb - dq2 * Lp;
    };
    // pressure: everything scales with P
    {
        const double iP = 1.0 / P;
        out.dP = core(A * iP, B * iP) + (Lb * o.q1 - o.q2 * Lp) * iP;
    }
    // temperature
    {
        double d[NC], td[NC], S = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double w = om[i];
            const double m = 0.480 + 1.574 * w - 0.176 * w * w;
            const double r = sqrt(T / Tc[i]);
            const double a = 1.0 + m * (1.0 - r);
            const double ap = -m * r / (2.0 * T);
            d[i] = ap / a - 1.0 / T;
            td[i] = e.s[i] * c[i] * d[i];
            S += td[i];
        }
        double chi[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) chi[i] = S;
#pragma unroll
        for (int i = 1; i < NC; ++i)
#pragma unroll
            for (int j = 0; j < i; ++j) {
                const double k = K[i * NC + j];
                chi[i] -= k * td[j];
                chi[j] -= k * td[i];
            }
        double dA = 0.0, lpsi = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double psi = e.s[i] * o.psi[i];
            dA += 2.0 * c[i] * d[i] * psi;
            lpsi += lam[i] * e.s[i] * (d[i] * o.psi[i] + chi[i]);
        }
        const double iT = 1.0 / T;
        out.dT = core(dA, -B * iT) - Lb * iT * o.q1 - o.q2 * lpsi;
    }
    // binary interaction parameters: per unit dA the change is Gam
    {
        const double Gam = core(1.0, 0.0);
        int q = 0;
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
            for (int b = a + 1; b < NC; ++b, ++q) {
                const double ss = e.s[a] * e.s[b];
                out.dk[q] = -2.0 * c[a] * c[b] * ss * Gam + o.q2 * ss * (lam[a] * c[b] + lam[b] * c[a]);
            }
    }
}

}  // namespace ptf
