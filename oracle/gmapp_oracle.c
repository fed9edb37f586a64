/*
 * gmapp_oracle.c -- plain FP64 CPU reference ("oracle") for the G-MAPP
 * multi-agent circular-field rollout (Bishnoi et al., "G-MAPP: GPU-accelerated
 * Multi-Agent Planning and Perception for Reactive Motion Generation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  It shares no code,
 * header, table or constant with the HIP library, and the library never calls it.
 *
 * Everything here is written for a reader holding the paper: one function per
 * equation, FP64 throughout (FP32 inputs are widened exactly by the caller),
 * no blocking, no fusion, no algebraic rewriting of the force law.  Agents are
 * independent, so the only parallelism is an OpenMP loop over agents.
 *
 * Readings where the paper is silent or ambiguous:
 *   - current vector (Eq. 3) parameterised by the agent's rotation vector:
 *     c = omega - n (n . omega), n the unit vector between agent and sphere centre;
 *   - clamped surface distance of Alg. 1: rho = max(|d| - (r_O + r_a), eps), used
 *     as the denominator of Eq. (2) and for the obstacle cost; k_f applied once;
 *   - cut-off of Alg. 1 (rho <= r_d), or a C1 smoothstep taper (cutoff = 1);
 *   - |w| = 0 gives no force; |d| = 0 gives n = 0;
 *   - explicit integrator: forces at step k use v^(k-1); Eq. (10) keeps its 1/2;
 *     Eq. (11) for a point mass is p^(k+1) = p^(k) + dt v^(k);
 *   - obstacles move with one constant velocity per segment inside the horizon.
 * Parity pins: see tests/test_oracle.py (closed forms, invariants, brute force).
 * Parity unpinned against the paper's own numbers: it prints no worked example.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* per-agent parameter row: k_a, d_a, k_f, r_d, r_a, omega_x, omega_y, omega_z */
enum { A_KA = 0, A_DA, A_KF, A_RD, A_RA, A_WX, A_WY, A_WZ, A_HEUR, A_N };
/* repulsive heuristic of an agent (Sec. III-A): circular field whose current is
 * parameterised by the agent's rotation vector, the same field with the current
 * taken from the relative velocity (Eq. 3 as printed), artificial potential field (Eq. 1) */
enum { H_CF_OMEGA = 0, H_MFI_VEL = 1, H_APF = 2 };
/* global parameter row */
enum { P_DT = 0, P_INVM, P_EPS, P_RC, P_W1, P_W2, P_W3, P_W4, P_AMAX, P_ALPHA, P_BAND, P_N };

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Cut-off weight sigma(rho): Alg. 1 keeps a sphere when rho <= r_d (hard).
 * cutoff == 1: C1 smoothstep taper over [r_d - band*r_d, r_d] (Sec. IV-A asks for
 * C1 potentials). */
double oracle_cutoff_weight(double rho, double r_d, int cutoff, double band)
{
    if (cutoff == 0) return rho <= r_d ? 1.0 : 0.0;
    double s = (r_d - rho) / (band * r_d);
    if (s <= 0.0) return 0.0;
    if (s >= 1.0) return 1.0;
    return s * s * (3.0 - 2.0 * s);
}

/* One agent-sphere interaction, Eq. (2) with the current vector of Eq. (3):
 *   d   = p - q                       (agent minus sphere centre)
 *   rho = max(|d| - R, eps)           (Alg. 1 surface distance, R = r_O + r_a)
 *   n   = d / |d|
 *   c   = omega - n (n . omega)       (current vector, orthogonal to n)
 *   f   = sigma(rho) (k_f / rho) (w/|w|) x (c x w),  w = relative velocity.
 * Returns rho through *rho_out. */
void oracle_pair_force(const double p[3], const double w[3], const double q[3], const double omega[3],
                       double k_f, double r_d, double R, double eps, int cutoff, double band,
                       double f[3], double *rho_out)
{
    double d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    double r = norm3(d);
    double rho = fmax(r - R, eps);
    *rho_out = rho;
    f[0] = f[1] = f[2] = 0.0;
    double sigma = oracle_cutoff_weight(rho, r_d, cutoff, band);
    if (sigma == 0.0) return;
    double n[3] = {0.0, 0.0, 0.0};
    if (r > 0.0) { n[0] = d[0] / r; n[1] = d[1] / r; n[2] = d[2] / r; }
    double nw = dot3(n, omega);
    double c[3] = {omega[0] - n[0] * nw, omega[1] - n[1] * nw, omega[2] - n[2] * nw};
    double wn = norm3(w);
    if (wn == 0.0) return;
    double u[3] = {w[0] / wn, w[1] / wn, w[2] / wn};
    double b[3], fu[3];
    cross3(c, w, b);
    cross3(u, b, fu);
    double s = sigma * k_f / rho;
    f[0] = s * fu[0]; f[1] = s * fu[1]; f[2] = s * fu[2];
}

/* Heuristic 2 with the current of Eq. (3) taken literally: c = w - n (n . w),
 * the relative velocity projected onto the surface; then Eq. (2) as above. */
static void mfi_vel_force(const double p[3], const double w[3], const double q[3], double k_f, double r_d, double R,
                          double eps, int cutoff, double band, double f[3], double *rho_out)
{
    oracle_pair_force(p, w, q, w, k_f, r_d, R, eps, cutoff, band, f, rho_out);
}

/* Heuristic 1 (APF, Eq. 1): f = k_f (1/rho - 1/r_d) (1/rho^2) n for a sphere within
 * the detection distance, n = d / |d| (d = p - q), with the distance to the sphere's
 * surface rho = max(|d| - R, eps) in place of |d| (the distance Eq. 1's condition
 * tests; FIRAS form).  The same cut-off weight as Eq. (2). */
void oracle_apf_force(const double p[3], const double q[3], double k_f, double r_d, double R, double eps, int cutoff,
                      double band, double f[3], double *rho_out)
{
    double d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
    double r = norm3(d);
    double rho = fmax(r - R, eps);
    *rho_out = rho;
    f[0] = f[1] = f[2] = 0.0;
    double sigma = oracle_cutoff_weight(rho, r_d, cutoff, band);
    if (sigma == 0.0 || r == 0.0) return;
    double mag = sigma * k_f * (1.0 / rho - 1.0 / r_d) / (rho * rho);
    f[0] = mag * d[0] / r; f[1] = mag * d[1] / r; f[2] = mag * d[2] / r;
}

/* The pair force of an agent with heuristic `heur`. */
void oracle_pair_force_h(int heur, const double p[3], const double w[3], const double q[3], const double omega[3],
                         double k_f, double r_d, double R, double eps, int cutoff, double band, double f[3],
                         double *rho_out)
{
    if (heur == H_APF) oracle_apf_force(p, q, k_f, r_d, R, eps, cutoff, band, f, rho_out);
    else if (heur == H_MFI_VEL) mfi_vel_force(p, w, q, k_f, r_d, R, eps, cutoff, band, f, rho_out);
    else oracle_pair_force(p, w, q, omega, k_f, r_d, R, eps, cutoff, band, f, rho_out);
}

/* segment (object) index of point j; -1 when the scene is static */
static int seg_of(long j, int n_seg, const int *seg_begin)
{
    for (int s = 0; s < n_seg; ++s)
        if (j >= seg_begin[s] && j < seg_begin[s + 1]) return s;
    return -1;
}

/* Repulsive force of Alg. 1 on one agent: the sum of Eq. (2) over every sphere of
 * S_W (Eq. 5) at time t, plus the minimum clamped surface distance over all
 * spheres (the distance of the obstacle cost, Eq. 18).  Sphere j sits at
 * q_j + t v_seg(j).  Diagnostics: sum of |f_j|; the pairs whose rho lies within
 * 1e-6 r_d of the hard cut-off (their classification may legitimately differ in
 * FP32); the sum of the magnitudes of the terms each pair force is made of, which
 * bounds what rounding can leave where terms cancel; and the sum of the force changes
 * when the agent's position in a moving segment's frame, p - t v_seg, is rounded to
 * FP32 (the position a single-precision evaluation works from).  Term magnitudes:
 *   circular fields, c = omega - n (n . omega) with omega = w for the velocity current:
 *     (k_f / rho) |w| (|omega| + |n . omega|) (Eqs. 2, 3: c x w and the projection cancel
 *     for motion along or across n);
 *   APF: k_f (1/rho + 1/r_d) / rho^2 (Eq. 1: 1/rho - 1/r_d cancels at the cut-off);
 *   both times sigma + |d sigma / d s| (rho + r_d) / (band r_d) under the taper, whose
 *   argument s = (r_d - rho) / (band r_d) cancels at its outer edge. */
static void repulsion_one(long n_pts, const double *px, const double *py, const double *pz, double r_obs,
                          int n_seg, const int *seg_begin, const double *seg_vel,
                          const double *ag, const double p[3], const double v[3], double t,
                          const double *prm, int cutoff,
                          double F[3], double *rho_min, double *abs_sum, double *edge_sum, long *edge_cnt,
                          double *term_sum, double *shift_sum)
{
    double omega[3] = {ag[A_WX], ag[A_WY], ag[A_WZ]};
    const int heur = (int)ag[A_HEUR];
    double R = r_obs + ag[A_RA];
    F[0] = F[1] = F[2] = 0.0;
    double rmin = INFINITY, asum = 0.0, esum = 0.0, tsum = 0.0, ssum = 0.0;
    const double r_d = ag[A_RD], band = prm[P_BAND];
    long ecnt = 0;
    for (long j = 0; j < n_pts; ++j) {
        int s = seg_of(j, n_seg, seg_begin);
        double vo[3] = {0.0, 0.0, 0.0};
        if (s >= 0) { vo[0] = seg_vel[3 * s]; vo[1] = seg_vel[3 * s + 1]; vo[2] = seg_vel[3 * s + 2]; }
        double q[3] = {px[j] + t * vo[0], py[j] + t * vo[1], pz[j] + t * vo[2]};
        double w[3] = {v[0] - vo[0], v[1] - vo[1], v[2] - vo[2]};
        double f[3], rho;
        oracle_pair_force_h(heur, p, w, q, omega, ag[A_KF], ag[A_RD], R, prm[P_EPS], cutoff, prm[P_BAND], f, &rho);
        F[0] += f[0]; F[1] += f[1]; F[2] += f[2];
        if (rho < rmin) rmin = rho;
        double fa = norm3(f);
        asum += fa;
        if (term_sum) {
            double weight = oracle_cutoff_weight(rho, r_d, cutoff, band);
            if (cutoff == 1) {
                const double st = (r_d - rho) / (band * r_d);
                if (st > 0.0 && st < 1.0) weight += 6.0 * st * (1.0 - st) * (rho + r_d) / (band * r_d);
            }
            if (heur == H_APF) {
                tsum += weight * ag[A_KF] * (1.0 / rho + 1.0 / r_d) / (rho * rho);
            } else {
                const double *om = heur == H_MFI_VEL ? w : omega;
                double d[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
                double r = norm3(d), nw = r > 0.0 ? dot3(d, om) / r : 0.0;
                tsum += weight * ag[A_KF] / rho * norm3(w) * (norm3(om) + fabs(nw));
            }
        }
        if (shift_sum && s >= 0) {
            /* the agent in the segment's frame, rounded to FP32, against the static point */
            double ps[3], q0[3] = {px[j], py[j], pz[j]}, fs[3], rs;
            for (int a = 0; a < 3; ++a) ps[a] = (double)(float)(p[a] - t * vo[a]);
            oracle_pair_force_h(heur, ps, w, q0, omega, ag[A_KF], r_d, R, prm[P_EPS], cutoff, band, fs, &rs);
            double df[3] = {fs[0] - f[0], fs[1] - f[1], fs[2] - f[2]};
            ssum += norm3(df);
        }
        if (edge_sum && cutoff == 0 && fabs(rho - ag[A_RD]) <= 1e-6 * ag[A_RD]) {
            ecnt += 1;
            /* the force such a pair would give if classified the other way */
            double fo[3], rr;
            oracle_pair_force_h(heur, p, w, q, omega, ag[A_KF], 2.0 * ag[A_RD] + 1.0, R, prm[P_EPS], 0, 0.0, fo,
                                &rr);
            esum += norm3(fo);
        }
    }
    *rho_min = rmin;
    if (abs_sum) *abs_sum = asum;
    if (edge_sum) *edge_sum = esum;
    if (edge_cnt) *edge_cnt = ecnt;
    if (term_sum) *term_sum = tsum;
    if (shift_sum) *shift_sum = ssum;
}

/* Teacher-forced force query (the response of Alg. 1 to one agent query), for a
 * batch of agents at given positions p[i], velocities v[i] and time t.
 * out rows per agent: F_r (3), rho_min, then (diagnostics != 0, else zeros) sum |f_j|, edge_force_sum,
 * edge_count, term magnitude sum, frame-rounding sum. */
int oracle_repulsion(long n_pts, const double *px, const double *py, const double *pz, double r_obs,
                     int n_seg, const int *seg_begin, const double *seg_vel,
                     int n_agents, const double *agents, const double *p, const double *v, double t,
                     const double *prm, int cutoff, int diagnostics, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_agents; ++i) {
        double F[3], rmin, asum = 0.0, esum = 0.0, tsum = 0.0, ssum = 0.0;
        long ecnt = 0;
        const int dg = diagnostics != 0;
        repulsion_one(n_pts, px, py, pz, r_obs, n_seg, seg_begin, seg_vel, agents + A_N * i, p + 3 * i,
                      v + 3 * i, t, prm, cutoff, F, &rmin, dg ? &asum : NULL, dg ? &esum : NULL,
                      dg ? &ecnt : NULL, dg ? &tsum : NULL, dg ? &ssum : NULL);
        double *o = out + 9 * i;
        o[0] = F[0]; o[1] = F[1]; o[2] = F[2]; o[3] = rmin; o[4] = asum; o[5] = esum; o[6] = (double)ecnt;
        o[7] = tsum; o[8] = ssum;
    }
    return 0;
}

/* Costs of Eqs. (16)-(20) for one trajectory p^(1..N) (pos: [N][3]) with the
 * per-step minimum obstacle distance rho_min^(k) (rmin: [N]).
 * out: C_goal, C_obs, C_path, C_smooth, C_total. */
void oracle_costs(int N, const double *pos, const double *rmin, const double goal[3], const double *prm,
                  double out[5])
{
    double rc = prm[P_RC], dt = prm[P_DT];
    double cg = 0.0, co = 0.0;
    for (int k = 0; k < N; ++k) {
        const double *pk = pos + 3 * k;
        double e[3] = {goal[0] - pk[0], goal[1] - pk[1], goal[2] - pk[2]};
        cg += fmin(norm3(e), rc) / rc;                   /* Eq. (17) */
        co += 1.0 - fmin(rmin[k], rc) / rc;              /* Eq. (18) */
    }
    cg /= N;
    co /= N;
    double L = 0.0;                                      /* path length, Eq. (19) */
    for (int k = 1; k < N; ++k) {
        double s[3] = {pos[3 * k] - pos[3 * k - 3], pos[3 * k + 1] - pos[3 * k - 2], pos[3 * k + 2] - pos[3 * k - 1]};
        L += norm3(s);
    }
    double e1[3] = {goal[0] - pos[0], goal[1] - pos[1], goal[2] - pos[2]};
    double d1 = norm3(e1);
    double cp;
    if (L >= d1) cp = (L > 0.0) ? 1.0 - d1 / L : 0.0;
    else cp = 1.0 - L / d1;
    double J = 0.0;                                      /* aggregate jerk, Eq. (20) */
    for (int k = 3; k < N; ++k) {
        double j3[3];
        for (int a = 0; a < 3; ++a)
            j3[a] = pos[3 * k + a] - 3.0 * pos[3 * (k - 1) + a] + 3.0 * pos[3 * (k - 2) + a] - pos[3 * (k - 3) + a];
        J += dot3(j3, j3);
    }
    double cs = fmin(1.0, J / ((double)N * dt * dt * dt * dt * prm[P_AMAX] * prm[P_AMAX]));
    out[0] = cg; out[1] = co; out[2] = cp; out[3] = cs;
    out[4] = prm[P_W1] * cg + prm[P_W2] * co + prm[P_W3] * cp + prm[P_W4] * cs;   /* Eq. (16) */
}

/* Selection rule: i* = argmin{C_i : C_i < alpha C_best}.  C_best is the cost of
 * the incumbent b this cycle; with no incumbent (b < 0) the plain argmin is taken.
 * Ties go to the lowest index; NaN costs never win. */
int oracle_select(int n, const double *total, int incumbent, double alpha)
{
    int best = -1;
    double bound = INFINITY;
    if (incumbent >= 0 && incumbent < n) bound = alpha * total[incumbent];
    for (int i = 0; i < n; ++i) {
        double c = total[i];
        if (!(c == c)) continue;
        if (incumbent >= 0 && incumbent < n && !(c < bound)) continue;
        if (best < 0 || c < total[best]) best = i;
    }
    if (best < 0 && incumbent >= 0 && incumbent < n) best = incumbent;
    return best;
}

/* One agent's forward rollout (Eqs. 6, 7, 9, 10, 11 for a point mass), with the
 * repulsive force of Alg. 1 at every step.
 * query: p0[3], v0[3], goal[3], t0 (time of step 1; moving spheres sit at p_j + t v_seg).
 * Records: pos [N+1][3] (p^(1..N+1)), vel [N+1][3] (v^(0..N)), rmin [N], force [N][3]
 * (F_r^(1..N)) and total force ftot [N][3] (F^(1..N)). */
static void rollout_one(long n_pts, const double *px, const double *py, const double *pz, double r_obs,
                        int n_seg, const int *seg_begin, const double *seg_vel, const double *ag,
                        const double *query, const double *prm, int N, int cutoff,
                        double *pos, double *vel, double *rmin, double *force, double *ftot)
{
    double p[3] = {query[0], query[1], query[2]};
    double v[3] = {query[3], query[4], query[5]};
    const double *g = query + 6;
    double dt = prm[P_DT], invm = prm[P_INVM];
    vel[0] = v[0]; vel[1] = v[1]; vel[2] = v[2];
    for (int k = 1; k <= N; ++k) {
        double t = query[9] + (k - 1) * dt;   /* cycle start time + step offset */
        double Fr[3], rho_min;
        repulsion_one(n_pts, px, py, pz, r_obs, n_seg, seg_begin, seg_vel, ag, p, v, t, prm, cutoff, Fr,
                      &rho_min, NULL, NULL, NULL, NULL, NULL);
        double F[3];
        for (int a = 0; a < 3; ++a)  /* Eq. (6) with the attractor of Eq. (7), e = p_g - p */
            F[a] = ag[A_KA] * (g[a] - p[a]) - ag[A_DA] * v[a] + Fr[a];
        double *pk = pos + 3 * (k - 1);
        pk[0] = p[0]; pk[1] = p[1]; pk[2] = p[2];
        rmin[k - 1] = rho_min;
        for (int a = 0; a < 3; ++a) {
            force[3 * (k - 1) + a] = Fr[a];
            ftot[3 * (k - 1) + a] = F[a];
            v[a] = v[a] + 0.5 * dt * invm * F[a];            /* Eqs. (9), (10) */
            p[a] = p[a] + dt * v[a];                           /* Eq. (11), point mass */
            vel[3 * k + a] = v[a];
        }
    }
    double *pe = pos + 3 * N;
    pe[0] = p[0]; pe[1] = p[1]; pe[2] = p[2];
}

/* Full planning cycle: rollout of every agent, costs, selection.
 * traj [Na][N+1][3], cost [Na][5], min_clear [Na][N] required;
 * force [Na][N][3], vel [Na][N+1][3], ftot [Na][N][3] optional (NULL). */
int oracle_rollout(long n_pts, const double *px, const double *py, const double *pz, double r_obs,
                   int n_seg, const int *seg_begin, const double *seg_vel,
                   int n_agents, const double *agents, const double *query, int incumbent,
                   const double *prm, int N, int cutoff,
                   double *traj, double *cost, double *min_clear, double *force, double *vel, double *ftot,
                   int *best)
{
    if (N < 1 || n_agents < 0 || n_pts < 0) return -1;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_agents; ++i) {
        double *fo = force ? force + (size_t)3 * N * i : malloc(sizeof(double) * 3 * N);
        double *vo = vel ? vel + (size_t)3 * (N + 1) * i : malloc(sizeof(double) * 3 * (N + 1));
        double *to = ftot ? ftot + (size_t)3 * N * i : malloc(sizeof(double) * 3 * N);
        if (!fo || !vo || !to) {
#pragma omp atomic write
            err = 1;
        } else {
            double *pos = traj + (size_t)3 * (N + 1) * i;
            double *rm = min_clear + (size_t)N * i;
            rollout_one(n_pts, px, py, pz, r_obs, n_seg, seg_begin, seg_vel, agents + A_N * i, query, prm, N,
                        cutoff, pos, vo, rm, fo, to);
            oracle_costs(N, pos, rm, query + 6, prm, cost + 5 * i);
        }
        if (!force) free(fo);
        if (!vel) free(vo);
        if (!ftot) free(to);
    }
    if (err) return -2;
    double *tot = malloc(sizeof(double) * (n_agents > 0 ? n_agents : 1));
    if (!tot) return -2;
    for (int i = 0; i < n_agents; ++i) tot[i] = cost[5 * i + 4];
    *best = oracle_select(n_agents, tot, incumbent, prm[P_ALPHA]);
    free(tot);
    return 0;
}
