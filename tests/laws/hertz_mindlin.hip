// Hertz-Mindlin with CoR damping, as a user law
__device__ void cdem_user_law(const double *n, double delta, const double *vrel, double Rbar, double mbar,
                              double estar, double gstar, double mu, double beta, double h,
                              const double *u_old, double *F, double *u_new) {
    const double kdamp = -2.0 * sqrt(5.0 / 6.0);
    double vn_s = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    double vn[3], vt[3];
    for (int i = 0; i < 3; i++) vn[i] = vn_s * n[i];
    for (int i = 0; i < 3; i++) vt[i] = vrel[i] - vn[i];
    double sq = sqrt(Rbar * delta);
    double Sn = 2.0 * estar * sq;
    double gn = kdamp * beta * sqrt(Sn * mbar);
    double kn = (4.0 / 3.0) * estar * sq * delta;
    double Fn[3];
    for (int i = 0; i < 3; i++) Fn[i] = kn * n[i] - gn * vn[i];
    double up[3];
    for (int i = 0; i < 3; i++) up[i] = u_old[i] + h * vt[i];
    double upn = up[0] * n[0] + up[1] * n[1] + up[2] * n[2];
    double ut[3];
    for (int i = 0; i < 3; i++) ut[i] = up[i] - upn * n[i];
    double St = 8.0 * gstar * sq;
    double gt = kdamp * beta * sqrt(St * mbar);
    double Ft[3];
    for (int i = 0; i < 3; i++) Ft[i] = -(St * ut[i]) - gt * vt[i];
    double fn_norm = sqrt(Fn[0] * Fn[0] + Fn[1] * Fn[1] + Fn[2] * Fn[2]);
    double ft_norm = sqrt(Ft[0] * Ft[0] + Ft[1] * Ft[1] + Ft[2] * Ft[2]);
    double cap = mu * fn_norm;
    if (ft_norm > cap) {
        double scale = cap / ft_norm;
        for (int i = 0; i < 3; i++) Ft[i] = Ft[i] * scale;
        double ut_norm = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
        if (ut_norm > 0.0) {
            double fac = (cap / St) / ut_norm;
            for (int i = 0; i < 3; i++) u_new[i] = fac * ut[i];
        } else {
            for (int i = 0; i < 3; i++) u_new[i] = 0.0;
        }
    } else {
        for (int i = 0; i < 3; i++) u_new[i] = ut[i];
    }
    for (int i = 0; i < 3; i++) F[i] = Fn[i] + Ft[i];
}
