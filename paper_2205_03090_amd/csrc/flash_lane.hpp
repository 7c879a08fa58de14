// flash_lane.hpp -- the per-mixture flash as a resumable state machine.
//
// One lane owns one mixture.  Each call of Lane::step() advances the mixture
// by one "step" whose expensive part is the same for every stage: up to two
// SRK phase evaluations (two compositions), optionally with composition
// derivatives, through single call sites, so that the lanes of a wavefront
// execute the equation of state together whatever stage each mixture is in.
// Stage-specific work (Rachford-Rice, convergence tests, acceleration,
// trust-region algebra, stage transitions) is cheap and runs before and
// after the evaluations.
//
// Stages and their two evaluation slots:
//   FEED      slot 0 = z                       -> d = ln z + ln phi(z)
//   PRE       slot 0 = x, slot 1 = y           initial substitutions + triage
//   SA        slot 0 = W^V, slot 1 = W^L       both stability trials together
//   SPLIT_SS  slot 0 = x, slot 1 = y           substitution of the split
//   SPLIT_NT  slot 0 = x, slot 1 = y (+ Phi)   trust region on G, refinement
//
// The method follows the paper's strategy (Sec. 2.2.3) with these readings:
//   * tm carries Michelsen's leading 1 (tm = 0 at the trivial point);
//   * Delta G of the triage is (1-theta) tpd(x) + theta tpd(y);
//   * a trial is unstable when tm < -eps_tm;
//   * dominant-eigenvalue acceleration at every dem_every-th substitution
//     update u >= 2: lambda = (s_u.s_u)/(s_{u-1}.s_u), extension by
//     s_u lambda/(1 - lambda) when 0 < lambda < 1, kept only if the
//     extrapolated point lowers the objective (tm, or G per unit feed),
//     otherwise replaced by the plain update (not counted as an iteration);
//   * the trials start from the Wilson K, the initial substitutions stop at
//     the first Rachford-Rice root outside (0,1) (case 1), and a case-3 split
//     continues from the latest K with a fresh substitution budget;
//   * the split trust region is scaled: u = D^(1/2) dn with
//     D = diag(z/(x y)), the paper's shift matrix;
//   * the converged split is refined by Newton steps until max |dn| is
//     below tol_polish, and y is chosen as the phase with the larger Z.
#pragma once

#include "srk_device.hpp"

namespace ptf {

enum Stage : int {
    ST_IDLE = 0,
    ST_FEED = 1,
    ST_PRE = 2,
    ST_SA = 3,
    ST_SPLIT_SS = 4,
    ST_SPLIT_NT = 5,
    ST_GONE = 6,
};

enum TrialMode : int { TM_SS = 0, TM_TR = 1, TM_DONE = 2 };

// A split whose smaller phase holds less than this fraction of the feed is
// reported as failed (single phase).
constexpr double kMinPhase = 1e-10;

// status bits (same values as the public header)
constexpr uint32_t kStInvalid = 0x0001u, kStShortcut = 0x0002u, kStSaRan = 0x0004u,
                   kStSaUnconv = 0x0008u, kStSplitTr = 0x0010u, kStSplitUnconv = 0x0020u,
                   kStSplitTrivial = 0x0040u, kStSplitFailed = 0x0080u,
                   kStRrNoRoot = 0x0100u, kStSwapped = 0x0200u, kStStepCap = 0x0400u;

// Kernel arguments shared by all forms.
struct FlashArgs {
    int64_t n;
    const double *z, *T, *P;
    int max_pre_ss, max_ss, max_tr_sa, max_tr_split, max_polish, dem_every, max_steps;
    int keep_factor;
    double tol_sa_ss, tol_sa_tr, tol_split_ss, tol_split_tr, tol_polish, eps_tm;
    int8_t *label;
    double *beta, *x, *y;
    int16_t *iters;
    uint16_t *status;
    uint32_t *flops;
    double *factor;
};

// Read-only shared component set (passed as separate restrict pointers so
// that compile-time indexed loads become wave-uniform scalar loads).
struct Props {
    const double *__restrict__ Tc;
    const double *__restrict__ Pc;
    const double *__restrict__ om;
    const double *__restrict__ K;
};

template <int NC>
struct Lane {
    static constexpr int NP = Tri<NC>::N;

    int stage;
    int64_t m;
    double T, P;
    double z[NC], d[NC];
    Eos<NC> e;
    // stage vectors:
    //   PRE/SPLIT_SS: v0 = ln K, v1 = previous substitution step
    //   SA:           v0 = ln W^V, v1 = ln W^L, v2/v3 = previous step (SS)
    //                 or accepted ln W (TR) of trial V / L
    //   SPLIT_NT:     v0 = n^V, v1 = accepted n^V
    double v0[NC], v1[NC], v2[NC], v3[NC];
    double theta;
    // stability trials
    int tmode[2];
    bool tpend[2];
    double trad[2], tfacc[2], tpred[2], tgacc[2], tmfin[2];
    // pending acceleration checks: objective before the extrapolation and
    // the extension applied (trials, split)
    bool tdem[2], sdem;
    double tmb[2], text[2], sgb, sext;
    // split trust region
    bool sinit, spend, spol;
    double srad, sfacc, spred, sgacc, sdprev;
    int it[8];
    uint32_t status, fl;
    int steps;

    __device__ __forceinline__ void start(int64_t mi, const FlashArgs &a, const Props &pr)
    {
        m = mi;
        stage = ST_FEED;
        T = a.T[mi];
        P = a.P[mi];
        status = 0;
        fl = 0;
        steps = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) it[k] = 0;
        double s = 0.0;
        bool ok = (T > 0.0) && (P > 0.0) && isfinite(T) && isfinite(P);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double zi = a.z[mi * NC + i];
            ok = ok && (zi > 0.0) && isfinite(zi);
            z[i] = zi;
            s += zi;
        }
        // shared set: Tc, Pc > 0, k symmetric with zero diagonal
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            ok = ok && (pr.Tc[i] > 0.0) && (pr.Pc[i] > 0.0) && isfinite(pr.om[i]);
            ok = ok && (pr.K[i * NC + i] == 0.0);
#pragma unroll
            for (int j = 0; j < i; ++j) ok = ok && (pr.K[i * NC + j] == pr.K[j * NC + i]);
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) z[i] = ok ? z[i] / s : z[i];
        if (!ok) {
            status = kStInvalid;
            finish_single(a);
            return;
        }
        eos_setup<NC>(e, pr.Tc, pr.Pc, pr.om, T, P);
    }

    __device__ __forceinline__ void wilson(double (&lk)[NC], const Props &pr) const
    {
#pragma unroll
        for (int i = 0; i < NC; ++i)
            lk[i] = log(pr.Pc[i] / P) + kWilson * (1.0 + pr.om[i]) * (1.0 - pr.Tc[i] / T);
    }

    __device__ __forceinline__ void write_counters(const FlashArgs &a)
    {
        if (a.iters) {
#pragma unroll
            for (int k = 0; k < 8; ++k) a.iters[m * 8 + k] = (int16_t)it[k];
        }
        if (a.status) a.status[m] = (uint16_t)status;
        if (a.flops) a.flops[m] = fl;
    }

    __device__ __forceinline__ void finish_single(const FlashArgs &a)
    {
        a.label[m] = 0;
        a.beta[m] = -1.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            a.x[m * NC + i] = z[i];
            a.y[m * NC + i] = z[i];
        }
        write_counters(a);
        stage = ST_IDLE;
    }

    // K -> Rachford-Rice -> normalised x, y (x_i = z_i/(1 + th(K_i - 1)),
    // y_i = K_i x_i).  False when no root exists.
    __device__ __forceinline__ bool xy_from_lnk(double (&x)[NC], double (&y)[NC],
                                                const double (&lnk)[NC])
    {
        double K[NC];
#pragma unroll
        for (int i = 0; i < NC; ++i) K[i] = exp(lnk[i]);
        fl += NC;
        if (!rr_solve<NC>(z, K, theta, fl)) return false;
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            x[i] = z[i] / (1.0 + theta * (K[i] - 1.0));
            y[i] = K[i] * x[i];
            sx += x[i];
            sy += y[i];
        }
        const double ix = 1.0 / sx, iy = 1.0 / sy;
#pragma unroll
        for (int i = 0; i < NC; ++i) { x[i] *= ix; y[i] *= iy; }
        fl += 8 * NC + 2;
        return true;
    }

    // x, y from the vapour mole numbers v0 = n^V: y = n^V/sum n^V,
    // x = (z - n^V)/sum(z - n^V).
    __device__ __forceinline__ void xy_from_nv(double (&x)[NC], double (&y)[NC], double &bv)
    {
        double sv = 0.0, sl = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            x[i] = z[i] - v0[i];
            y[i] = v0[i];
            sv += y[i];
            sl += x[i];
        }
        const double iv = 1.0 / sv, il = 1.0 / sl;
#pragma unroll
        for (int i = 0; i < NC; ++i) { x[i] *= il; y[i] *= iv; }
        bv = sv;
        fl += 5 * NC + 2;
    }

    __device__ __forceinline__ void enter_sa(const Props &pr)
    {
        double lk[NC];
        wilson(lk, pr);
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double lz = log(z[i]);
            v0[i] = lz + lk[i];
            v1[i] = lz - lk[i];
        }
        fl += 8 * NC;
        stage = ST_SA;
        status |= kStSaRan;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            tmode[t] = TM_SS;
            tpend[t] = false;
            trad[t] = 0.0;
            tmfin[t] = 0.0;
            tdem[t] = false;
        }
    }

    __device__ __forceinline__ void enter_split_ss()
    {
        stage = ST_SPLIT_SS;
        theta = 0.5;
        sdem = false;
    }

    // One substitution update with acceleration: v += s (1 + ext), where s
    // is the plain step and ext the dominant-eigenvalue extension when the
    // update index u is a multiple of dem_every.
    __device__ __forceinline__ double ss_update(double (&v)[NC], double (&prev)[NC],
                                                const double (&s)[NC], int u, int dem)
    {
        double ext = 0.0;
        if (dem > 0 && u >= 2 && (u % dem) == 0) {
            double num = 0.0, den = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) { num += s[i] * s[i]; den += prev[i] * s[i]; }
            const double lam = num / den;
            if (lam > 0.0 && lam < 1.0) ext = lam / (1.0 - lam);
            fl += 4 * NC + 3;
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            v[i] += s[i] + ext * s[i];
            prev[i] = s[i];
        }
        fl += 3 * NC;
        return ext;
    }

    // ------------------------------------------------------------------
    // Prepare: choose the compositions of the two evaluation slots.
    // ------------------------------------------------------------------
    __device__ __forceinline__ void prepare(double (&w0)[NC], double (&w1)[NC], bool &e0,
                                            bool &e1, bool &p0, bool &p1, const FlashArgs &a,
                                            const Props &pr)
    {
        e0 = e1 = p0 = p1 = false;
        if (stage == ST_FEED) {
#pragma unroll
            for (int i = 0; i < NC; ++i) w0[i] = z[i];
            e0 = true;
            return;
        }
        if (stage == ST_PRE) {
            if (xy_from_lnk(w0, w1, v0) && theta > 0.0 && theta < 1.0) {
                e0 = e1 = true;
                return;
            }
            enter_sa(pr);   // case 1: theta left (0,1)
        }
        if (stage == ST_SA) {
            if (tmode[0] != TM_DONE) {
#pragma unroll
                for (int i = 0; i < NC; ++i) w0[i] = exp(v0[i]);
                e0 = true;
                p0 = (tmode[0] == TM_TR) || (it[1] == a.max_ss);
                fl += NC;
            }
            if (tmode[1] != TM_DONE) {
#pragma unroll
                for (int i = 0; i < NC; ++i) w1[i] = exp(v1[i]);
                e1 = true;
                p1 = (tmode[1] == TM_TR) || (it[3] == a.max_ss);
                fl += NC;
            }
            return;
        }
        if (stage == ST_SPLIT_SS) {
            if (xy_from_lnk(w0, w1, v0)) {
                e0 = e1 = true;
                return;
            }
            status |= kStRrNoRoot | kStSplitFailed;
            finish_single(a);
            return;
        }
        if (stage == ST_SPLIT_NT) {
            double bv;
            if (!sinit) {
                double x[NC], y[NC];
                if (!xy_from_lnk(x, y, v0) || !(theta > 0.0 && theta < 1.0)) {
                    status |= kStSplitFailed;
                    finish_single(a);
                    return;
                }
#pragma unroll
                for (int i = 0; i < NC; ++i) v0[i] = theta * y[i];
                sinit = true;
            }
            xy_from_nv(w0, w1, bv);
            e0 = e1 = p0 = p1 = true;
        }
    }

    // ------------------------------------------------------------------
    // Stability trial T at its evaluation (Sec. 2.2.1; Appendix B.1).
    // F holds the derivatives Phi on entry (when havephi) and is reused for
    // the Cholesky factor.
    // ------------------------------------------------------------------
    template <int TR>
    __device__ __forceinline__ void sa_consume(const Phase<NC> &o, const double (&W)[NC],
                                               bool havephi, const FlashArgs &a,
                                               double (&F)[NP], double (&Hs)[NP],
                                               double (&dinv)[NC])
    {
        double(&lw)[NC] = TR == 0 ? v0 : v1;
        double(&aux)[NC] = TR == 0 ? v2 : v3;
        int &ss = it[TR == 0 ? 1 : 3];
        int &tr = it[TR == 0 ? 2 : 4];
        double grad[NC], tm = 1.0, sw = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            grad[i] = lw[i] + o.lnphi[i] - d[i];
            tm += W[i] * (grad[i] - 1.0);
            sw += W[i];
        }
        fl += 6 * NC;
        if (tmode[TR] == TM_SS) {
            double gmax = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) gmax = fmax(gmax, fabs(grad[i]));
            if (tm < -a.eps_tm || gmax < a.tol_sa_ss) {
                tmode[TR] = TM_DONE;
                tmfin[TR] = tm;
                return;
            }
            if (tdem[TR]) {
                // an extrapolated point is kept only if it lowers tm
                tdem[TR] = false;
                if (!(tm < tmb[TR])) {
#pragma unroll
                    for (int i = 0; i < NC; ++i) lw[i] -= text[TR] * aux[i];
                    return;   // evaluate the plain update instead
                }
            }
            if (ss < a.max_ss) {
                double st[NC];
#pragma unroll
                for (int i = 0; i < NC; ++i) st[i] = -grad[i];
                const double ext = ss_update(lw, aux, st, ss + 1, a.dem_every);
                ++ss;
                if (ext > 0.0) {
                    tdem[TR] = true;
                    tmb[TR] = tm;
                    text[TR] = ext;
                }
                return;
            }
            // substitution budget spent: the trust region starts at this
            // point (its derivatives were requested for this evaluation)
            tmode[TR] = TM_TR;
            tpend[TR] = false;
            trad[TR] = 0.0;
        }
        // ---- trust region in beta = 2 sqrt(W) ----
        double g[NC], gmax = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            g[i] = sqrt(W[i]) * grad[i];
            gmax = fmax(gmax, fabs(g[i]));
        }
        fl += 3 * NC;
        if (tpend[TR]) {
            tpend[TR] = false;
            const double pred = tpred[TR];
            bool accept;
            double ratio = 1.0;
            if (fabs(pred) < 1e-13) {
                accept = gmax < tgacc[TR];
            } else {
                ratio = (tm - tfacc[TR]) / pred;
                accept = (tm < tfacc[TR]) && ratio > 0.0;
            }
            if (!accept) {
                trad[TR] *= 0.5;
#pragma unroll
                for (int i = 0; i < NC; ++i) lw[i] = aux[i];
                return;   // re-evaluate at the accepted point
            }
            if (ratio <= 0.25) trad[TR] *= 0.5;
            else if (ratio >= 0.75) trad[TR] *= 2.0;
        }
        // at an accepted point
        if (tm < -a.eps_tm || gmax < a.tol_sa_tr) {
            tmode[TR] = TM_DONE;
            tmfin[TR] = tm;
            return;
        }
        if (tr >= a.max_tr_sa) {
            tmode[TR] = TM_DONE;
            tmfin[TR] = tm;
            status |= kStSaUnconv;
            return;
        }
        if (!havephi) return;   // derivatives arrive with the next evaluation
        // H_ij = delta_ij (1 + g_i/beta_i) + sqrt(W_i W_j) d ln phi_i/d W_j
        //      = delta_ij (1 + grad_i/2) + sqrt(c_i c_j) Phi_ij     (eq. analysis_hess)
        double rc[NC];
        const double isw = 1.0 / sw;
#pragma unroll
        for (int i = 0; i < NC; ++i) rc[i] = sqrt(W[i] * isw);
#pragma unroll
        for (int i = 0; i < NC; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j)
                Hs[tri(i, j)] = rc[i] * rc[j] * F[tri(i, j)] + ((i == j) ? 1.0 + 0.5 * grad[i] : 0.0);
        fl += 2 * NP + 4 * NC;
        double u[NC];
        bool eta0;
        double pred = trust_step<NC>(u, trad[TR], eta0, F, dinv, Hs, g, fl);
        // keep beta positive (fraction to the boundary)
        double amax = 1.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const double bi = 2.0 * sqrt(W[i]);
            if (u[i] < 0.0) amax = fmin(amax, 0.99 * bi / -u[i]);
        }
        if (amax < 1.0) {
            double gu = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) gu += g[i] * u[i];
            pred = amax * gu + amax * amax * (pred - gu);
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            aux[i] = lw[i];
            lw[i] = 2.0 * log(sqrt(W[i]) + 0.5 * amax * u[i]);
        }
        fl += 6 * NC;
        tfacc[TR] = tm;
        tgacc[TR] = gmax;
        tpred[TR] = pred;
        tpend[TR] = true;
        ++tr;
    }

    // Both trials done: label decision and K re-estimate (Sec. 2.2.1).
    __device__ __forceinline__ void sa_finish(const FlashArgs &a)
    {
        const bool unstable = (tmfin[0] < -a.eps_tm) || (tmfin[1] < -a.eps_tm);
        if (!unstable) {
            finish_single(a);
            return;
        }
        if (tmfin[1] < tmfin[0]) {
#pragma unroll
            for (int i = 0; i < NC; ++i) v0[i] = log(z[i]) - v1[i];
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i) v0[i] = v0[i] - log(z[i]);
        }
        fl += 2 * NC;
        enter_split_ss();
    }

    // Two-phase result from n^V (v0), canonical orientation by Z.
    __device__ __forceinline__ void finish_two(const FlashArgs &a, double zx, double zy,
                                               const double (&Lf)[NP], bool savef,
                                               const double (&vs)[NC])
    {
        double x[NC], y[NC], bv;
        xy_from_nv(x, y, bv);
        double lk = 0.0;
#pragma unroll
        for (int i = 0; i < NC; ++i) lk = fmax(lk, fabs(log(y[i] / x[i])));
        if (!(bv > kMinPhase && bv < 1.0 - kMinPhase)) {
            status |= kStSplitFailed;
            finish_single(a);
            return;
        }
        if (lk < 1e-6) {
            status |= kStSplitTrivial;
            finish_single(a);
            return;
        }
        const bool swap = zx > zy;
        if (swap) status |= kStSwapped;
        a.label[m] = 1;
        a.beta[m] = swap ? 1.0 - bv : bv;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            a.x[m * NC + i] = swap ? y[i] : x[i];
            a.y[m * NC + i] = swap ? x[i] : y[i];
        }
        if (a.keep_factor && a.factor) {
            // factor of H~ = D^(1/2) H' D^(1/2): row i of L' scaled by 1/v_i
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j)
                    a.factor[m * NP + tri(i, j)] = savef ? Lf[tri(i, j)] / vs[i] : NAN;
        }
        write_counters(a);
        stage = ST_IDLE;
    }

    // ------------------------------------------------------------------
    // One step.
    // ------------------------------------------------------------------
    __device__ __forceinline__ void step(const FlashArgs &a, const Props &pr)
    {
        if (stage == ST_IDLE || stage == ST_GONE) return;
        if (++steps > a.max_steps) {
            status |= kStStepCap;
            finish_single(a);
            return;
        }
        double w0[NC], w1[NC];
        bool e0, e1, p0, p1;
        prepare(w0, w1, e0, e1, p0, p1, a, pr);
        if (stage == ST_IDLE) return;

        // F: derivatives Phi of the current slot, then the Cholesky factor
        double F[NP], Hs[NP], dinv[NC];
        Phase<NC> o;
        const bool split_nt = (stage == ST_SPLIT_NT);
        // split trust region (scaled by v_i = sqrt(x_i y_i / z_i)):
        //   H' = (I - v v' + V((1-th) Phi^V + th Phi^L) V) / (th (1-th)),
        // accumulated across the two slots (liquid slot first).
        double vs[NC], bvap = 0.0;
        if (split_nt) {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                bvap += v0[i];
                vs[i] = sqrt(w0[i] * w1[i] / z[i]);
            }
            fl += 4 * NC;
        }

        // ---------------- slot 0 ----------------
        if (e0) phase_eval<NC>(o, e, pr.K, w0, fl);
        if (p0) phase_derivs<NC>(F, o, e, pr.K, fl);
        if (stage == ST_SA && e0 && tmode[0] != TM_DONE)
            sa_consume<0>(o, w0, p0, a, F, Hs, dinv);
        if (split_nt) {
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j) Hs[tri(i, j)] = bvap * vs[i] * vs[j] * F[tri(i, j)];
            fl += 3 * NP;
        }
        // keep what the consumers need from slot 0
        double r0[NC];
        const double Z0 = o.Z;
#pragma unroll
        for (int i = 0; i < NC; ++i) r0[i] = o.lnphi[i];

        // ---------------- slot 1 ----------------
        if (e1) phase_eval<NC>(o, e, pr.K, w1, fl);
        if (p1) phase_derivs<NC>(F, o, e, pr.K, fl);
        if (stage == ST_SA && e1 && tmode[1] != TM_DONE)
            sa_consume<1>(o, w1, p1, a, F, Hs, dinv);

        // ---------------- consume ----------------
        if (stage == ST_FEED) {
#pragma unroll
            for (int i = 0; i < NC; ++i) d[i] = log(z[i]) + r0[i];
            fl += 2 * NC;
            wilson(v0, pr);
            fl += 5 * NC;
            theta = 0.5;
            stage = ST_PRE;
            return;
        }
        if (stage == ST_PRE) {
#pragma unroll
            for (int i = 0; i < NC; ++i) v0[i] = r0[i] - o.lnphi[i];
            fl += NC;
            ++it[0];
            if (it[0] < a.max_pre_ss) return;
            // triage (Sec. 2.2.3): tpd of the current liquid and vapour
            double tx = 0.0, ty = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                tx += w0[i] * (log(w0[i]) + r0[i] - d[i]);
                ty += w1[i] * (log(w1[i]) + o.lnphi[i] - d[i]);
            }
            const double dg = (1.0 - theta) * tx + theta * ty;
            fl += 8 * NC + 3;
            if (tx < -a.eps_tm || ty < -a.eps_tm || dg < -a.eps_tm) {
                status |= kStShortcut;
                enter_split_ss();
            } else {
                enter_sa(pr);
            }
            return;
        }
        if (stage == ST_SA) {
            if (tmode[0] == TM_DONE && tmode[1] == TM_DONE) sa_finish(a);
            return;
        }
        if (stage == ST_SPLIT_SS) {
            int &ss = it[5];
            // G per unit feed (eq. gibbs) where an acceleration check needs it
            const bool dem_next = a.dem_every > 0 && ss + 1 >= 2 && ((ss + 1) % a.dem_every) == 0;
            double G = 0.0;
            if (sdem || dem_next) {
#pragma unroll
                for (int i = 0; i < NC; ++i)
                    G += (1.0 - theta) * w0[i] * (log(w0[i]) + r0[i]) +
                         theta * w1[i] * (log(w1[i]) + o.lnphi[i]);
                fl += 10 * NC;
            }
            if (sdem) {
                // an extrapolated point is kept only if it lowers G
                sdem = false;
                if (!(G < sgb)) {
#pragma unroll
                    for (int i = 0; i < NC; ++i) v0[i] -= sext * v1[i];
                    return;   // evaluate the plain update instead
                }
            }
            double st[NC], dmax = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                st[i] = (r0[i] - o.lnphi[i]) - v0[i];
                dmax = fmax(dmax, fabs(exp(st[i]) - 1.0));
            }
            fl += 4 * NC;
            const double ext = ss_update(v0, v1, st, ss + 1, a.dem_every);
            ++ss;
            if (!(dmax < a.tol_split_ss) && ss < a.max_ss && ext > 0.0) {
                sdem = true;
                sgb = G;
                sext = ext;
            }
            if (dmax < a.tol_split_ss || ss >= a.max_ss) {
                if (!(dmax < a.tol_split_ss)) status |= kStSplitTr;
                stage = ST_SPLIT_NT;
                sinit = false;
                spend = false;
                spol = false;
                srad = 0.0;
            }
            return;
        }
        if (stage == ST_SPLIT_NT) {
            const double th = bvap;
            // gradient of G over n^V (eq. split_grad) and G itself (eq. gibbs)
            double gt[NC], gs[NC], G = 0.0, gmax = 0.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const double fx = log(w0[i]) + r0[i];
                const double fy = log(w1[i]) + o.lnphi[i];
                gt[i] = fy - fx;
                G += (z[i] - v0[i]) * fx + v0[i] * fy;
                gmax = fmax(gmax, fabs(gt[i]));
                gs[i] = vs[i] * gt[i];
            }
            fl += 11 * NC;
            const double sc = 1.0 / (th * (1.0 - th));
#pragma unroll
            for (int i = 0; i < NC; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j) {
                    double h = Hs[tri(i, j)] + (1.0 - th) * vs[i] * vs[j] * F[tri(i, j)]
                               - vs[i] * vs[j];
                    if (i == j) h += 1.0;
                    Hs[tri(i, j)] = h * sc;
                }
            fl += 8 * NP;
            if (spend) {
                spend = false;
                bool accept;
                double ratio = 1.0;
                if (fabs(spred) < 1e-13) {
                    accept = gmax < sgacc;
                } else {
                    ratio = (G - sfacc) / spred;
                    accept = (G < sfacc) && ratio > 0.0;
                }
                if (!accept) {
                    srad *= 0.5;
#pragma unroll
                    for (int i = 0; i < NC; ++i) v0[i] = v1[i];
                    return;   // re-evaluate at the accepted point
                }
                if (ratio <= 0.25) srad *= 0.5;
                else if (ratio >= 0.75) srad *= 2.0;
            }
            if (!spol && gmax < a.tol_split_tr) {
                spol = true;   // the paper's criterion holds: refine
                sdprev = 1e300;
            }
            double u[NC];
            bool eta0;
            if (spol) {
                // Newton refinement: the unshifted step while H is positive
                // definite; an indefinite H sends the split back to the trust
                // region
                double rad = 1e300;
                trust_step<NC>(u, rad, eta0, F, dinv, Hs, gs, fl);
                if (!eta0) spol = false;
            }
            if (spol) {
                double dmax = 0.0, amax = 1.0;
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                    u[i] *= vs[i];
                    dmax = fmax(dmax, fabs(u[i]));
                    if (u[i] < 0.0) amax = fmin(amax, 0.99 * v0[i] / -u[i]);
                    if (u[i] > 0.0) amax = fmin(amax, 0.99 * (z[i] - v0[i]) / u[i]);
                }
#pragma unroll
                for (int i = 0; i < NC; ++i) v0[i] += amax * u[i];
                fl += 6 * NC;
                // converged: step below tol_polish, or steps of rounding size
                // that no longer shrink
                const bool conv = dmax < a.tol_polish || (dmax < 1e-10 && dmax >= 0.5 * sdprev);
                if (conv || it[7] >= a.max_polish) {
                    if (!conv && !(dmax < 1e-10)) status |= kStSplitUnconv;
                    finish_two(a, Z0, o.Z, F, true, vs);
                    return;
                }
                sdprev = dmax;
                ++it[7];
                return;
            }
            if (it[6] >= a.max_tr_split) {
                status |= kStSplitUnconv;
                finish_two(a, Z0, o.Z, F, false, vs);
                return;
            }
            status |= kStSplitTr;
            double pred = trust_step<NC>(u, srad, eta0, F, dinv, Hs, gs, fl);
            // dn = v o u, kept inside 0 < n^V < z
            double amax = 1.0;
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                u[i] *= vs[i];
                if (u[i] < 0.0) amax = fmin(amax, 0.99 * v0[i] / -u[i]);
                if (u[i] > 0.0) amax = fmin(amax, 0.99 * (z[i] - v0[i]) / u[i]);
            }
            if (amax < 1.0) {
                double gu = 0.0;
#pragma unroll
                for (int i = 0; i < NC; ++i) gu += gt[i] * u[i];
                pred = amax * gu + amax * amax * (pred - gu);
            }
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                v1[i] = v0[i];
                v0[i] += amax * u[i];
            }
            fl += 6 * NC;
            sfacc = G;
            sgacc = gmax;
            spred = pred;
            spend = true;
            ++it[6];
            return;
        }
    }
};

}  // namespace ptf
