/* FP64 oracle for 6-D pose agents -- TEST INFRASTRUCTURE ONLY.
 *
 * A pose agent moves in Spin(3) x| R^3 (Sec. II) by Eqs. (6)-(11) of Sec. IV-A:
 * the wrench F = K e - D v + (0, f_r) with e = log(M^-1 M_g), the twist update
 * v += (dt/2) I F and the pose update M <- M exp(dt v).  Rotations are held as
 * 3x3 matrices built from unit quaternions; exp and log are the Lie-group maps
 * of SE(3) written out from their definitions:
 *   exp(phi, rho) = (Rot(phi), J(phi) rho)
 *   log(R, t)     = (phi, J(phi)^-1 t), phi the rotation vector of R (angle <= pi)
 *   J(phi) = I + (1 - cos th)/th^2 [phi] + (th - sin th)/th^3 [phi]^2
 * with the inverse of J taken by solving the 3x3 system (Gaussian elimination),
 * not by a closed form, so that it checks the device's closed form.  Twists and
 * wrenches are in the body frame (omega, u); the repulsive force of Alg. 1 is
 * evaluated at the agent's position with its world velocity R u and rotated into
 * the body frame.  Costs are those of Eqs. (16)-(20) on the positions.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* from gmapp_oracle.c */
int oracle_repulsion(long n_pts, const double *px, const double *py, const double *pz, double r_obs, int n_seg,
                     const int *seg_begin, const double *seg_vel, int n_agents, const double *agents,
                     const double *p, const double *v, double t, const double *prm, int cutoff, int diagnostics,
                     double *out);
void oracle_costs(int N, const double *pos, const double *rmin, const double goal[3], const double *prm,
                  double out[5]);
int oracle_select(int n, const double *total, int incumbent, double alpha);

enum { A_KA = 0, A_DA = 1, A_N = 9 };          /* agent row layout of gmapp_oracle.c */
enum { P_DT = 0, P_INVM = 1, P_ALPHA = 9 };    /* parameter row layout of gmapp_oracle.c */

typedef double M3[3][3];

static void quat_to_mat(const double q_in[4], M3 R)
{
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

/* the unit quaternion (w >= 0) of a rotation matrix, from its largest diagonal combination */
static void mat_to_quat(M3 R, double q[4])
{
    double tr = R[0][0] + R[1][1] + R[2][2];
    double w, x, y, z;
    if (tr > 0) {
        double s = 2.0 * sqrt(1.0 + tr);
        w = 0.25 * s; x = (R[2][1] - R[1][2]) / s; y = (R[0][2] - R[2][0]) / s; z = (R[1][0] - R[0][1]) / s;
    } else if (R[0][0] > R[1][1] && R[0][0] > R[2][2]) {
        double s = 2.0 * sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]);
        w = (R[2][1] - R[1][2]) / s; x = 0.25 * s; y = (R[0][1] + R[1][0]) / s; z = (R[0][2] + R[2][0]) / s;
    } else if (R[1][1] > R[2][2]) {
        double s = 2.0 * sqrt(1.0 + R[1][1] - R[0][0] - R[2][2]);
        w = (R[0][2] - R[2][0]) / s; x = (R[0][1] + R[1][0]) / s; y = 0.25 * s; z = (R[1][2] + R[2][1]) / s;
    } else {
        double s = 2.0 * sqrt(1.0 + R[2][2] - R[0][0] - R[1][1]);
        w = (R[1][0] - R[0][1]) / s; x = (R[0][2] + R[2][0]) / s; y = (R[1][2] + R[2][1]) / s; z = 0.25 * s;
    }
    double n = sqrt(w * w + x * x + y * y + z * z);
    if (w < 0) n = -n;
    q[0] = w / n; q[1] = x / n; q[2] = y / n; q[3] = z / n;
}

static void mat_mul(M3 A, M3 B, M3 C)
{
    M3 T;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[i][j] = A[i][0] * B[0][j] + A[i][1] * B[1][j] + A[i][2] * B[2][j];
    memcpy(C, T, sizeof(M3));
}

static void mat_vec(M3 A, const double v[3], double o[3])
{
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[i][0] * v[0] + A[i][1] * v[1] + A[i][2] * v[2];
    o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
}

static void mat_tvec(M3 A, const double v[3], double o[3])   /* A^T v */
{
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[0][i] * v[0] + A[1][i] * v[1] + A[2][i] * v[2];
    o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
}

static void skew(const double p[3], M3 S)
{
    S[0][0] = 0; S[0][1] = -p[2]; S[0][2] = p[1];
    S[1][0] = p[2]; S[1][1] = 0; S[1][2] = -p[0];
    S[2][0] = -p[1]; S[2][1] = p[0]; S[2][2] = 0;
}

/* Rodrigues: Rot(phi) = I + sin th / th [phi] + (1 - cos th) / th^2 [phi]^2 */
static void so3_exp(const double phi[3], M3 R)
{
    double th = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    double a = th < 1e-8 ? 1.0 - th * th / 6.0 : sin(th) / th;
    double b = th < 1e-8 ? 0.5 - th * th / 24.0 : (1.0 - cos(th)) / (th * th);
    M3 S, S2;
    skew(phi, S);
    mat_mul(S, S, S2);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = (i == j) + a * S[i][j] + b * S2[i][j];
}

/* rotation vector of R, angle in [0, pi] (via the quaternion, w >= 0) */
static void so3_log(M3 R, double phi[3])
{
    double q[4];
    mat_to_quat(R, q);
    double n = sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double f = n < 1e-15 ? 2.0 / q[0] : 2.0 * atan2(n, q[0]) / n;
    phi[0] = f * q[1]; phi[1] = f * q[2]; phi[2] = f * q[3];
}

static void left_jacobian(const double phi[3], M3 J)
{
    double th = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    double a = th < 1e-5 ? 0.5 - th * th / 24.0 : (1.0 - cos(th)) / (th * th);
    double b = th < 1e-5 ? 1.0 / 6.0 - th * th / 120.0 : (th - sin(th)) / (th * th * th);
    M3 S, S2;
    skew(phi, S);
    mat_mul(S, S, S2);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[i][j] = (i == j) + a * S[i][j] + b * S2[i][j];
}

/* solve J x = t by Gaussian elimination with partial pivoting */
static void solve3(M3 J_in, const double t[3], double x[3])
{
    double A[3][4];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) A[i][j] = J_in[i][j];
        A[i][3] = t[i];
    }
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        for (int j = 0; j < 4; ++j) { double tmp = A[c][j]; A[c][j] = A[piv][j]; A[piv][j] = tmp; }
        for (int r = c + 1; r < 3; ++r) {
            double f = A[r][c] / A[c][c];
            for (int j = c; j < 4; ++j) A[r][j] -= f * A[c][j];
        }
    }
    for (int r = 2; r >= 0; --r) {
        double s = A[r][3];
        for (int j = r + 1; j < 3; ++j) s -= A[r][j] * x[j];
        x[r] = s / A[r][r];
    }
}

/* SE(3) maps, exported for the pins: quaternion (w >= 0) + translation */
void oracle_se3_exp(const double phi[3], const double rho[3], double q[4], double t[3])
{
    M3 R, J;
    so3_exp(phi, R);
    left_jacobian(phi, J);
    mat_to_quat(R, q);
    mat_vec(J, rho, t);
}

void oracle_se3_log(const double q[4], const double t[3], double phi[3], double rho[3])
{
    M3 R, J;
    quat_to_mat(q, R);
    so3_log(R, phi);
    left_jacobian(phi, J);
    solve3(J, t, rho);
}

/* One pose agent over N steps.  query: p0, v0 (world), goal, t0; pq: q0[4], w0[3]
 * (body), qg[4]; gains: k_r, d_r, i_r.  Records pos [N+1][3], rot [N+1][4] (w >= 0),
 * rmin [N]. */
static void rollout_pose_one(long n_pts, const double *px, const double *py, const double *pz, double r_obs,
                             int n_seg, const int *seg_begin, const double *seg_vel, const double *ag,
                             const double *gains, const double *query, const double *pq, const double *prm, int N,
                             int cutoff, double *pos, double *rot, double *rmin)
{
    M3 R, Rg;
    quat_to_mat(pq, R);
    quat_to_mat(pq + 7, Rg);
    double p[3] = {query[0], query[1], query[2]};
    double om[3] = {pq[4], pq[5], pq[6]};
    double u[3];
    mat_tvec(R, query + 3, u);                       /* body linear velocity */
    const double *g = query + 6;
    double dt = prm[P_DT], invm = prm[P_INVM];
    double kr = gains[0], dr = gains[1], ir = gains[2];
    for (int k = 1; k <= N; ++k) {
        double t = query[9] + (k - 1) * dt;
        double vw[3], out[9];
        mat_vec(R, u, vw);                           /* world velocity of the body origin */
        oracle_repulsion(n_pts, px, py, pz, r_obs, n_seg, seg_begin, seg_vel, 1, ag, p, vw, t, prm, cutoff, 0, out);
        memcpy(pos + 3 * (k - 1), p, sizeof(p));
        mat_to_quat(R, rot + 4 * (k - 1));
        rmin[k - 1] = out[3];
        /* e = log(M^-1 M_g): M^-1 M_g = (R^T R_g, R^T (p_g - p)) */
        M3 Re, Rt;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Rt[i][j] = R[j][i];
        mat_mul(Rt, Rg, Re);
        double te[3] = {g[0] - p[0], g[1] - p[1], g[2] - p[2]}, phi_e[3], rho_e[3], fb[3];
        mat_tvec(R, te, te);
        M3 Je;
        so3_log(Re, phi_e);
        left_jacobian(phi_e, Je);
        solve3(Je, te, rho_e);
        mat_tvec(R, out, fb);                        /* f_r in the body frame */
        double Fa[3], Fl[3];
        for (int a = 0; a < 3; ++a) {                /* Eqs. (6), (7) */
            Fa[a] = kr * phi_e[a] - dr * om[a];
            Fl[a] = ag[A_KA] * rho_e[a] - ag[A_DA] * u[a] + fb[a];
        }
        for (int a = 0; a < 3; ++a) {                /* Eqs. (9), (10) */
            om[a] += 0.5 * dt * ir * Fa[a];
            u[a] += 0.5 * dt * invm * Fl[a];
        }
        /* Eq. (11): M <- M exp(dt v) */
        double dphi[3] = {dt * om[0], dt * om[1], dt * om[2]}, drho[3] = {dt * u[0], dt * u[1], dt * u[2]};
        M3 dR, dJ;
        so3_exp(dphi, dR);
        left_jacobian(dphi, dJ);
        double dtr[3], dw[3];
        mat_vec(dJ, drho, dtr);
        mat_vec(R, dtr, dw);
        for (int a = 0; a < 3; ++a) p[a] += dw[a];
        mat_mul(R, dR, R);
    }
    memcpy(pos + 3 * N, p, sizeof(p));
    mat_to_quat(R, rot + 4 * N);
}

/* Planning cycle of pose agents: rollouts, costs (on the positions), selection.
 * gains: [Na][3] (k_r, d_r, i_r); pq: q0[4], w0[3], qg[4]. */
int oracle_rollout_pose(long n_pts, const double *px, const double *py, const double *pz, double r_obs, int n_seg,
                        const int *seg_begin, const double *seg_vel, int n_agents, const double *agents,
                        const double *gains, const double *query, const double *pq, int incumbent,
                        const double *prm, int N, int cutoff, double *traj, double *rot, double *cost,
                        double *min_clear, int *best)
{
    if (N < 1 || n_agents < 0 || n_pts < 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n_agents; ++i) {
        double *pos = traj + (size_t)3 * (N + 1) * i;
        double *rm = min_clear + (size_t)N * i;
        rollout_pose_one(n_pts, px, py, pz, r_obs, n_seg, seg_begin, seg_vel, agents + A_N * i, gains + 3 * i,
                         query, pq, prm, N, cutoff, pos, rot + (size_t)4 * (N + 1) * i, rm);
        oracle_costs(N, pos, rm, query + 6, prm, cost + 5 * i);
    }
    double *tot = malloc(sizeof(double) * (n_agents > 0 ? n_agents : 1));
    if (!tot) return -2;
    for (int i = 0; i < n_agents; ++i) tot[i] = cost[5 * i + 4];
    *best = oracle_select(n_agents, tot, incumbent, prm[P_ALPHA]);
    free(tot);
    return 0;
}
