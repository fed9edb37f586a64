/*
 * gmapp_oracle_grad.c -- FP64 forward-mode (dual-number) reference gradient of
 * each agent's total cost C_i (Eq. 16) with respect to its own parameters
 * theta_i = (k_a, d_a, k_f, omega_x, omega_y, omega_z).
 *
 * TEST INFRASTRUCTURE ONLY (see gmapp_oracle.c).  The rollout below is the one of
 * gmapp_oracle.c carried out in dual numbers: every value travels with its six
 * partial derivatives, so the derivative is exact up to FP64 rounding wherever
 * the rollout is differentiable (the hard cut-off of Alg. 1 is not; gradients are
 * meant for the C1 taper, cutoff = 1).  Agents are independent, so dC_i/dtheta_j = 0
 * for i != j and only the diagonal blocks are computed.
 * Pinned by central finite differences of the plain FP64 oracle (tests/test_oracle.py).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ND 6
typedef struct { double v; double d[ND]; } dual;

enum { A_KA = 0, A_DA, A_KF, A_RD, A_RA, A_WX, A_WY, A_WZ, A_HEUR, A_N };   /* rotation-vector field only */
enum { P_DT = 0, P_INVM, P_EPS, P_RC, P_W1, P_W2, P_W3, P_W4, P_AMAX, P_ALPHA, P_BAND, P_N };

static dual dc(double v) { dual r; r.v = v; memset(r.d, 0, sizeof r.d); return r; }
static dual dvar(double v, int k) { dual r = dc(v); r.d[k] = 1.0; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
static dual dmul(dual a, dual b)
{
    dual r; r.v = a.v * b.v;
    for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
static dual ddiv(dual a, dual b)
{
    dual r; r.v = a.v / b.v;
    for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return r;
}
static dual ddivc(dual a, double c) { dual b = {c, {0}}; return ddiv(a, b); }
static dual dscale(dual a, double s) { dual r; r.v = a.v * s; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * s; return r; }
static dual dsqrt(dual a)
{
    dual r; r.v = sqrt(a.v);
    for (int k = 0; k < ND; ++k) r.d[k] = (r.v > 0.0) ? a.d[k] / (2.0 * r.v) : 0.0;
    return r;
}
static dual dmin(dual a, dual b) { return (b.v < a.v) ? b : a; }
static dual dmax(dual a, dual b) { return (b.v > a.v) ? b : a; }
static dual ddot3(const dual a[3], const dual b[3]) { return dadd(dadd(dmul(a[0], b[0]), dmul(a[1], b[1])), dmul(a[2], b[2])); }
static void dcross3(const dual a[3], const dual b[3], dual o[3])
{
    o[0] = dsub(dmul(a[1], b[2]), dmul(a[2], b[1]));
    o[1] = dsub(dmul(a[2], b[0]), dmul(a[0], b[2]));
    o[2] = dsub(dmul(a[0], b[1]), dmul(a[1], b[0]));
}

static dual cutoff_weight(dual rho, double r_d, int cutoff, double band)
{
    if (cutoff == 0) return dc(rho.v <= r_d ? 1.0 : 0.0);
    dual s = ddivc(dsub(dc(r_d), rho), band * r_d);
    if (s.v <= 0.0) return dc(0.0);
    if (s.v >= 1.0) return dc(1.0);
    return dmul(dmul(s, s), dsub(dc(3.0), dscale(s, 2.0)));
}

/* Eq. (2) with the current vector of Eq. (3) (same readings as gmapp_oracle.c). */
static void pair_force(const dual p[3], const dual w[3], const double q[3], const dual omega[3], dual k_f,
                       double r_d, double R, double eps, int cutoff, double band, dual f[3], dual *rho_out)
{
    dual d[3] = {dsub(p[0], dc(q[0])), dsub(p[1], dc(q[1])), dsub(p[2], dc(q[2]))};
    dual r = dsqrt(ddot3(d, d));
    dual rho = dmax(dsub(r, dc(R)), dc(eps));
    *rho_out = rho;
    f[0] = f[1] = f[2] = dc(0.0);
    dual sigma = cutoff_weight(rho, r_d, cutoff, band);
    if (sigma.v == 0.0) return;
    dual n[3] = {dc(0.0), dc(0.0), dc(0.0)};
    if (r.v > 0.0) { n[0] = ddiv(d[0], r); n[1] = ddiv(d[1], r); n[2] = ddiv(d[2], r); }
    dual nw = ddot3(n, omega);
    dual c[3] = {dsub(omega[0], dmul(n[0], nw)), dsub(omega[1], dmul(n[1], nw)), dsub(omega[2], dmul(n[2], nw))};
    dual wn = dsqrt(ddot3(w, w));
    if (wn.v == 0.0) return;
    dual u[3] = {ddiv(w[0], wn), ddiv(w[1], wn), ddiv(w[2], wn)};
    dual b[3], fu[3];
    dcross3(c, w, b);
    dcross3(u, b, fu);
    dual s = ddiv(dmul(sigma, k_f), rho);
    f[0] = dmul(s, fu[0]); f[1] = dmul(s, fu[1]); f[2] = dmul(s, fu[2]);
}

static int seg_of(long j, int n_seg, const int *seg_begin)
{
    for (int s = 0; s < n_seg; ++s)
        if (j >= seg_begin[s] && j < seg_begin[s + 1]) return s;
    return -1;
}

static dual dnorm3(const dual a[3]) { return dsqrt(ddot3(a, a)); }

/* Costs of Eqs. (16)-(20) in dual numbers (pos: [N][3] = p^(1..N)). */
static dual costs(int N, const dual *pos, const dual *rmin, const double goal[3], const double *prm, dual out[4])
{
    double rc = prm[P_RC], dt = prm[P_DT];
    dual cg = dc(0.0), co = dc(0.0);
    for (int k = 0; k < N; ++k) {
        dual e[3] = {dsub(dc(goal[0]), pos[3 * k]), dsub(dc(goal[1]), pos[3 * k + 1]), dsub(dc(goal[2]), pos[3 * k + 2])};
        cg = dadd(cg, ddivc(dmin(dnorm3(e), dc(rc)), rc));
        co = dadd(co, dsub(dc(1.0), ddivc(dmin(rmin[k], dc(rc)), rc)));
    }
    cg = ddivc(cg, (double)N);
    co = ddivc(co, (double)N);
    dual L = dc(0.0);
    for (int k = 1; k < N; ++k) {
        dual s[3] = {dsub(pos[3 * k], pos[3 * k - 3]), dsub(pos[3 * k + 1], pos[3 * k - 2]), dsub(pos[3 * k + 2], pos[3 * k - 1])};
        L = dadd(L, dnorm3(s));
    }
    dual e1[3] = {dsub(dc(goal[0]), pos[0]), dsub(dc(goal[1]), pos[1]), dsub(dc(goal[2]), pos[2])};
    dual d1 = dnorm3(e1);
    dual cp;
    if (L.v >= d1.v) cp = (L.v > 0.0) ? dsub(dc(1.0), ddiv(d1, L)) : dc(0.0);
    else cp = dsub(dc(1.0), ddiv(L, d1));
    dual J = dc(0.0);
    for (int k = 3; k < N; ++k) {
        dual j3[3];
        for (int a = 0; a < 3; ++a)
            j3[a] = dsub(dadd(dsub(pos[3 * k + a], dscale(pos[3 * (k - 1) + a], 3.0)), dscale(pos[3 * (k - 2) + a], 3.0)),
                         pos[3 * (k - 3) + a]);
        J = dadd(J, ddot3(j3, j3));
    }
    dual cs = dmin(dc(1.0), ddivc(J, (double)N * dt * dt * dt * dt * prm[P_AMAX] * prm[P_AMAX]));
    out[0] = cg; out[1] = co; out[2] = cp; out[3] = cs;
    return dadd(dadd(dadd(dscale(cg, prm[P_W1]), dscale(co, prm[P_W2])), dscale(cp, prm[P_W3])), dscale(cs, prm[P_W4]));
}

/* grad [Na][7]: C_i followed by dC_i/d(k_a, d_a, k_f, omega_x, omega_y, omega_z). */
int oracle_rollout_grad(long n_pts, const double *px, const double *py, const double *pz, double r_obs,
                        int n_seg, const int *seg_begin, const double *seg_vel,
                        int n_agents, const double *agents, const double *query,
                        const double *prm, int N, int cutoff, double *grad)
{
    if (N < 1 || n_agents < 0 || n_pts < 0) return -1;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_agents; ++i) {
        const double *ag = agents + A_N * i;
        dual *pos = malloc(sizeof(dual) * 3 * (size_t)N);
        dual *rmin = malloc(sizeof(dual) * (size_t)N);
        if (!pos || !rmin) {
#pragma omp atomic write
            err = 1;
            free(pos); free(rmin);
            continue;
        }
        dual ka = dvar(ag[A_KA], 0), da = dvar(ag[A_DA], 1), kf = dvar(ag[A_KF], 2);
        dual omega[3] = {dvar(ag[A_WX], 3), dvar(ag[A_WY], 4), dvar(ag[A_WZ], 5)};
        double R = r_obs + ag[A_RA];
        double dt = prm[P_DT], invm = prm[P_INVM];
        const double *g = query + 6;
        dual p[3] = {dc(query[0]), dc(query[1]), dc(query[2])};
        dual v[3] = {dc(query[3]), dc(query[4]), dc(query[5])};
        for (int k = 1; k <= N; ++k) {
            double t = query[9] + (k - 1) * dt;
            dual Fr[3] = {dc(0.0), dc(0.0), dc(0.0)};
            dual rm = dc(INFINITY);
            for (long j = 0; j < n_pts; ++j) {
                int s = seg_of(j, n_seg, seg_begin);
                double vo[3] = {0.0, 0.0, 0.0};
                if (s >= 0) { vo[0] = seg_vel[3 * s]; vo[1] = seg_vel[3 * s + 1]; vo[2] = seg_vel[3 * s + 2]; }
                double q[3] = {px[j] + t * vo[0], py[j] + t * vo[1], pz[j] + t * vo[2]};
                dual w[3] = {dsub(v[0], dc(vo[0])), dsub(v[1], dc(vo[1])), dsub(v[2], dc(vo[2]))};
                dual f[3], rho;
                pair_force(p, w, q, omega, kf, ag[A_RD], R, prm[P_EPS], cutoff, prm[P_BAND], f, &rho);
                Fr[0] = dadd(Fr[0], f[0]); Fr[1] = dadd(Fr[1], f[1]); Fr[2] = dadd(Fr[2], f[2]);
                rm = dmin(rm, rho);
            }
            dual F[3];
            for (int a = 0; a < 3; ++a)
                F[a] = dadd(dsub(dmul(ka, dsub(dc(g[a]), p[a])), dmul(da, v[a])), Fr[a]);
            for (int a = 0; a < 3; ++a) pos[3 * (k - 1) + a] = p[a];
            rmin[k - 1] = rm;
            for (int a = 0; a < 3; ++a) {
                v[a] = dadd(v[a], dscale(F[a], 0.5 * dt * invm));
                p[a] = dadd(p[a], dscale(v[a], dt));
            }
        }
        dual parts[4];
        dual C = costs(N, pos, rmin, g, prm, parts);
        double *o = grad + 7 * i;
        o[0] = C.v;
        for (int k = 0; k < ND; ++k) o[1 + k] = C.d[k];
        free(pos);
        free(rmin);
    }
    return err ? -2 : 0;
}
