// Host-side discretisation and partition tables of the truncated additive
// overlapping DDM (Leng & Ju, Sec. 2.2 and Sec. 3.1), built once per problem.
//
// Conventions (the paper states them in the continuum):
//  * per axis, unknowns at nodes g = -n_pml+1 .. M+n_pml-1, Dirichlet beyond;
//    PML profile sigma0 (t/n_pml)^2, t = cells outside [0, M];
//  * half-open cores [iC, (i+1)C-1], the outer ones holding the global PML;
//  * every interior side extended by n_ov overlap cells (sigma = 0, the shifted
//    profile of eq. PMLprofile) plus n_pml PML cells, Dirichlet at n_ov+n_pml;
//  * cut-off factor at node offset m outside a core: 1 (m <= 1),
//    beta0((m-1)/(n_ov-1)) (1 < m < n_ov), 0 (m >= n_ov), with the quintic
//    smoothstep beta0(t) = 1 - t^3 (10 - 15 t + 6 t^2), monotone and C^2 as
//    Sec. 2.2 requires.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>

#include "ddm_internal.h"

namespace ddm {

namespace {

using cd = std::complex<double>;

struct AxisGeom {
    int M, N, C, n_pml, n_ov;
    double s0;
    int clo(int i) const { return i == 0 ? -n_pml + 1 : i * C; }
    int chi(int i) const { return i == N - 1 ? M + n_pml - 1 : (i + 1) * C - 1; }
    int lo(int i) const { return i == 0 ? clo(i) : clo(i) - (n_ov + n_pml - 1); }
    int hi(int i) const { return i == N - 1 ? chi(i) : chi(i) + (n_ov + n_pml - 1); }
    double profile(double cells_past) const {  // sigma0 (t/n_pml)^2, t >= 0
        double t = cells_past > 0 ? cells_past : 0.0;
        return s0 * (t / n_pml) * (t / n_pml);
    }
    double sigma_global(double x) const {
        if (x < 0) return profile(-x);
        if (x > M) return profile(x - M);
        return 0.0;
    }
    // Subdomain i's truncated problem: shifted profile past n_ov overlap cells
    // on interior sides, the global profile elsewhere.
    double sigma_sub(int i, double x) const {
        if (i > 0 && x < clo(i)) return profile(clo(i) - x - n_ov);
        if (i < N - 1 && x > chi(i)) return profile(x - chi(i) - n_ov);
        return sigma_global(x);
    }
};

Coef make_coef(double s_mid, double s_plus, double s_minus, double h) {
    cd a0(1.0, s_mid), ap(1.0, s_plus), am(1.0, s_minus);
    cd cp = 1.0 / (a0 * ap * h * h);
    cd cm = 1.0 / (a0 * am * h * h);
    Coef c;
    c.cp = make_double2(cp.real(), cp.imag());
    c.cm = make_double2(cm.real(), cm.imag());
    return c;
}

double beta0(double t) {
    if (t <= 0) return 1.0;
    if (t >= 1) return 0.0;
    return 1.0 - t * t * t * (10.0 - 15.0 * t + 6.0 * t * t);
}

}  // namespace

int build_plan(const ddm_problem *p, Plan *plan, std::string *err) {
    char buf[256];
    if (!p) { *err = "null problem"; return DDM_EINVAL; }
    if (p->dim != 2 && p->dim != 3) { *err = "dim must be 2 or 3"; return DDM_EINVAL; }
    if (!(p->h > 0) || !std::isfinite(p->h)) { *err = "h must be positive and finite"; return DDM_EINVAL; }
    if (!(p->sigma0 >= 0) || !std::isfinite(p->sigma0)) { *err = "sigma0 must be >= 0 and finite"; return DDM_EINVAL; }
    if (p->n_pml < 2) { *err = "n_pml must be >= 2"; return DDM_EINVAL; }
    if (p->n_ov < 2) { *err = "n_ov must be >= 2"; return DDM_EINVAL; }
    Plan &P = *plan;
    P = Plan();
    P.dim = p->dim;
    P.n_pml = p->n_pml;
    P.n_ov = p->n_ov;
    P.h = p->h;
    P.sigma0 = p->sigma0;
    P.nsub = 1;
    AxisGeom ax[3];
    for (int d = 0; d < 3; ++d) {
        if (d < p->dim) {
            if (p->M[d] < 1 || p->N[d] < 1 || p->M[d] % p->N[d] != 0) {
                snprintf(buf, sizeof buf, "axis %d: M=%d must be a positive multiple of N=%d", d, p->M[d], p->N[d]);
                *err = buf;
                return DDM_EINVAL;
            }
            int C = p->M[d] / p->N[d];
            if (p->N[d] > 1 && C < p->n_ov + 2) {
                snprintf(buf, sizeof buf, "axis %d: core width %d < n_ov + 2 = %d", d, C, p->n_ov + 2);
                *err = buf;
                return DDM_EINVAL;
            }
            P.M[d] = p->M[d];
            P.N[d] = p->N[d];
            P.C[d] = C;
            P.G[d] = p->M[d] + 2 * p->n_pml - 1;
            P.glo[d] = -p->n_pml + 1;
        } else {
            P.M[d] = 0; P.N[d] = 1; P.C[d] = 1; P.G[d] = 1; P.glo[d] = 0;
        }
        ax[d] = AxisGeom{P.M[d], P.N[d], P.C[d], p->n_pml, p->n_ov, p->sigma0};
        P.nsub *= P.N[d];
    }
    P.nglob = (long long)P.G[0] * P.G[1] * P.G[2];
    P.ring = p->dim == 2 ? 3 : 4;

    // global coefficient tables
    for (int d = 0; d < 3; ++d) {
        P.gcoff[d] = (int)P.gcoef.size();
        for (int gi = 0; gi < P.G[d]; ++gi) {
            double x = P.glo[d] + gi;
            if (d < p->dim)
                P.gcoef.push_back(make_coef(ax[d].sigma_global(x), ax[d].sigma_global(x + 0.5),
                                            ax[d].sigma_global(x - 0.5), p->h));
            else
                P.gcoef.push_back(Coef{make_double2(0, 0), make_double2(0, 0)});
        }
    }

    // subdomains
    long long off = 0, foff = 0;
    P.subs.resize(P.nsub);
    for (int a = 0; a < P.nsub; ++a) {
        SubDesc &s = P.subs[a];
        int id[3] = {a % P.N[0], (a / P.N[0]) % P.N[1], a / (P.N[0] * P.N[1])};
        long long cnt = 1;
        for (int d = 0; d < 3; ++d) {
            s.sid[d] = id[d];
            if (d < p->dim) {
                s.clo[d] = ax[d].clo(id[d]);
                s.chi[d] = ax[d].chi(id[d]);
                s.lo[d] = ax[d].lo(id[d]);
                s.hi[d] = ax[d].hi(id[d]);
            } else {
                s.clo[d] = s.chi[d] = s.lo[d] = s.hi[d] = 0;
            }
            s.n[d] = s.hi[d] - s.lo[d] + 1;
            cnt *= s.n[d];
        }
        s.nloc = cnt;
        s.off = off;
        off += cnt;
        s.nb = s.n[p->dim - 1];
        s.bs = (int)(cnt / s.nb);
        s.ld = (p->precision == DDM_MIXED && (s.bs & 1)) ? s.bs + 1 : s.bs;
        {
            const int grp = p->precision == DDM_MIXED ? 8 : 4;
            s.mpad = s.bs <= kMmaMaxBs ? (s.bs + grp - 1) / grp * grp : 0;
        }
        s.foff = foff;
        // room for either layout of the inverses (column-major with stride ld,
        // or the matrix-core order with mpad columns), so the substitution
        // variant can change without a new allocation
        foff += (long long)s.nb * s.bs * std::max(s.ld, s.mpad);
        if (s.mpad > P.mpad_max) P.mpad_max = s.mpad;
        if (s.bs > P.bs_max) P.bs_max = s.bs;
        if (s.nb > P.nb_max) P.nb_max = s.nb;
        for (int d = 0; d < 3; ++d) {
            s.coff[d] = (int)P.coef.size();
            for (int x = 0; x < s.n[d]; ++x) {
                double g = s.lo[d] + x;
                if (d < p->dim)
                    P.coef.push_back(make_coef(ax[d].sigma_sub(id[d], g), ax[d].sigma_sub(id[d], g + 0.5),
                                               ax[d].sigma_sub(id[d], g - 0.5), p->h));
                else
                    P.coef.push_back(Coef{make_double2(0, 0), make_double2(0, 0)});
            }
        }
        int k = 0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0 && dz == 0) continue;
                    int nid[3] = {id[0] + dx, id[1] + dy, id[2] + dz};
                    bool ok = true;
                    for (int d = 0; d < 3; ++d)
                        if (nid[d] < 0 || nid[d] >= P.N[d]) ok = false;
                    s.nbr[k] = ok ? nid[0] + P.N[0] * (nid[1] + P.N[1] * nid[2]) : -1;
                    s.lag[k] = (dx != 0) + (dy != 0) + (dz != 0);
                    ++k;
                }
        for (int r0 = 0; r0 < s.bs; r0 += 64) P.items.push_back(SolveItem{a, r0});
    }
    P.etot = off;
    P.fel = foff;
    P.w_el_by_l.assign(P.nb_max, 0.0);
    P.v_el_by_l.assign(P.nb_max, 0.0);
    for (const SubDesc &s : P.subs)
        for (int l = 0; l < s.nb; ++l) {
            P.w_el_by_l[l] += (double)s.bs * s.bs;
            P.v_el_by_l[l] += (double)s.bs;
        }
    // two chains per subdomain (both-ends elimination) while they all fit on
    // the device's compute units (one 1024-thread chain workgroup per CU) and
    // the chain kernel applies (block size <= 256), one otherwise
    plan_set_twist(&P, plan_twist_fits(P));
    P.btab.resize(p->n_ov + 1);
    for (int m = 0; m <= p->n_ov; ++m)
        P.btab[m] = m <= 1 ? 1.0 : (m >= p->n_ov ? 0.0 : beta0((double)(m - 1) / (double)(p->n_ov - 1)));
    // transfer strips: nodes of a box within the first or last n_ov core
    // layers along some axis (only there can a neighbour's transfer be
    // non-zero)
    for (int a = 0; a < P.nsub; ++a) {
        const SubDesc &sd = P.subs[a];
        for (long long e = 0; e < sd.nloc; ++e) {
            const int l[3] = {(int)(e % sd.n[0]), (int)((e / sd.n[0]) % sd.n[1]), (int)(e / ((long long)sd.n[0] * sd.n[1]))};
            bool in = false;
            for (int d = 0; d < p->dim; ++d) {
                const int x = sd.lo[d] + l[d];
                if (x >= sd.clo[d] && x <= sd.clo[d] + p->n_ov - 1) in = true;
                if (x <= sd.chi[d] && x >= sd.chi[d] - p->n_ov + 1) in = true;
            }
            if (in) P.strip.push_back(make_int2(a, (int)e));
        }
    }
    // assembly tables: per axis and global index, the boxes whose cut-off
    // b(m) is non-zero there (the factor of eq. tsum along that axis)
    auto side = [&](int m) { return m <= 1 ? 1.0 : (m >= p->n_ov ? 0.0 : P.btab[m]); };
    for (int d = 0; d < 3; ++d) {
        P.aoff[d] = (int)P.aown.size();
        for (int gi = 0; gi < P.G[d]; ++gi) {
            AxisOwn e{};
            if (d >= p->dim) {
                e.beta[0] = 1.0;
                e.n[0] = 1;
                e.cnt = 1;
            } else {
                const int x = P.glo[d] + gi;
                for (int i = 0; i < P.N[d]; ++i) {
                    if (x < ax[d].lo(i) || x > ax[d].hi(i)) continue;
                    double b = 1.0;
                    if (x > ax[d].chi(i)) b = side(x - ax[d].chi(i));
                    else if (x < ax[d].clo(i)) b = side(ax[d].clo(i) - x);
                    if (b == 0.0) continue;
                    if (e.cnt == 2) {
                        *err = "more than two boxes with a non-zero cut-off at one node";
                        return DDM_EINVAL;
                    }
                    e.beta[e.cnt] = b;
                    e.i[e.cnt] = i;
                    e.lc[e.cnt] = x - ax[d].lo(i);
                    e.n[e.cnt] = ax[d].hi(i) - ax[d].lo(i) + 1;
                    ++e.cnt;
                }
            }
            P.aown.push_back(e);
        }
    }
    return DDM_OK;
}

bool plan_twist_fits(const Plan &P) { return 2 * P.nsub <= P.ncu && P.nb_max >= 4 && P.bs_max <= 256; }

void plan_set_twist(Plan *plan, bool twisted) {
    plan->twisted = twisted;
    for (SubDesc &s : plan->subs) s.mid = twisted ? s.nb / 2 : s.nb - 1;
}

}  // namespace ddm
