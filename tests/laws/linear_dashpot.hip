// Linear spring-dashpot contact (no friction): F = (k delta - c v_n) n with a
// constant stiffness k and the damping c = 2 zeta sqrt(k mbar) of a fixed
// damping ratio zeta; the tangential history stays zero.
__device__ void cdem_user_law(const double *n, double delta, const double *vrel, double Rbar, double mbar,
                              double estar, double gstar, double mu, double beta, double h,
                              const double *u_old, double *F, double *u_new) {
    const double k = 1.0e3, zeta = 0.05;
    const double c = 2.0 * zeta * sqrt(k * mbar);
    const double vn = vrel[0] * n[0] + vrel[1] * n[1] + vrel[2] * n[2];
    const double f = k * delta - c * vn;
    for (int i = 0; i < 3; i++) {
        F[i] = f * n[i];
        u_new[i] = 0.0;
    }
}
