// 1-D reference operators of the DGSEM (Sec. 3.1.1), computed on the host in FP64.
//
// Gauss-Legendre nodes: roots of P_{N+1} by Newton's method from the
// asymptotic guesses cos(pi (i + 3/4) / (N + 3/2)); weights 2 / ((1 - x^2) P'(x)^2).
// Gauss-Lobatto nodes: +-1 and the roots of P_N' (Newton on P_N' using the
// Legendre equation for P_N''); weights 2 / (N (N + 1) P_N(x)^2).
// Lagrange derivative at the nodes from barycentric weights; the weak-form
// derivative matrix of the collocated DGSEM is
//   Dhat[i][lam] = -(omega_lam / omega_i) l_i'(xi_lam),
// (the weight ratio the weak form produces; free-stream and polynomial
// exactness hold with it), and lhat_i(+-1) = l_i(+-1) / omega_i.  For the BR2
// lifting of the Navier-Stokes equations also the strong-form derivative
// Dstr[i][lam] = l_lam'(xi_i) and the face values built from it.
#include <cmath>
#include "hbpc_internal.hpp"

static void legendre(int n, double x, double& p, double& dp) {
    // P_n(x) and P_n'(x) by the three-term recurrence
    double p0 = 1.0, p1 = x;
    if (n == 0) { p = 1.0; dp = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    p = p1;
    // P_n' = n (x P_n - P_{n-1}) / (x^2 - 1), away from +-1
    if (std::fabs(std::fabs(x) - 1.0) < 1e-300) dp = 0.5 * n * (n + 1.0) * (x > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0));
    else dp = n * (x * p1 - p0) / (x * x - 1.0);
}

bool basis1d_build(int N, int kind, Basis1DHost& B) {
    const int NP = N + 1;
    B.N = N;
    B.NP = NP;
    B.xi.assign(NP, 0.0);
    B.w.assign(NP, 0.0);
    const double pi = 3.14159265358979323846;
    if (kind == HBPC_NODES_GAUSS) {
        for (int i = 0; i < NP; ++i) {
            double x = -std::cos(pi * (i + 0.75) / (NP + 0.5));
            for (int it = 0; it < 100; ++it) {
                double p, dp;
                legendre(NP, x, p, dp);
                double dx = p / dp;
                x -= dx;
                if (std::fabs(dx) < 1e-16) break;
            }
            double p, dp;
            legendre(NP, x, p, dp);
            B.xi[i] = x;
            B.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
        }
    } else if (kind == HBPC_NODES_LOBATTO) {
        if (N < 1) return false;
        B.xi[0] = -1.0;
        B.xi[N] = 1.0;
        for (int i = 1; i < N; ++i) {
            double x = -std::cos(pi * i / N);
            for (int it = 0; it < 100; ++it) {
                double p, dp;
                legendre(N, x, p, dp);
                double d2p = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
                double dx = dp / d2p;
                x -= dx;
                if (std::fabs(dx) < 1e-16) break;
            }
            B.xi[i] = x;
        }
        for (int i = 0; i < NP; ++i) {
            double p, dp;
            legendre(N, B.xi[i], p, dp);
            B.w[i] = 2.0 / (N * (N + 1.0) * p * p);
        }
    } else {
        return false;
    }
    // barycentric weights
    std::vector<double> bw(NP, 1.0);
    for (int i = 0; i < NP; ++i)
        for (int j = 0; j < NP; ++j)
            if (j != i) bw[i] /= (B.xi[i] - B.xi[j]);
    // Dstd[lam][i] = l_i'(xi_lam)
    std::vector<double> Dstd(NP * NP, 0.0);
    for (int lam = 0; lam < NP; ++lam) {
        double diag = 0.0;
        for (int i = 0; i < NP; ++i) {
            if (i == lam) continue;
            double v = (bw[i] / bw[lam]) / (B.xi[lam] - B.xi[i]);
            Dstd[lam * NP + i] = v;
            diag -= v;
        }
        Dstd[lam * NP + lam] = diag;
    }
    B.Dhat.assign(NP * NP, 0.0);
    for (int i = 0; i < NP; ++i)
        for (int lam = 0; lam < NP; ++lam) B.Dhat[i * NP + lam] = -(B.w[lam] / B.w[i]) * Dstd[lam * NP + i];
    // boundary values of the Lagrange basis
    B.lp.assign(NP, 0.0);
    B.lm.assign(NP, 0.0);
    for (int i = 0; i < NP; ++i) {
        double a = 1.0, b = 1.0;
        for (int j = 0; j < NP; ++j) {
            if (j == i) continue;
            a *= (1.0 - B.xi[j]) / (B.xi[i] - B.xi[j]);
            b *= (-1.0 - B.xi[j]) / (B.xi[i] - B.xi[j]);
        }
        B.lp[i] = a;
        B.lm[i] = b;
    }
    B.lhp.resize(NP);
    B.lhm.resize(NP);
    for (int i = 0; i < NP; ++i) {
        B.lhp[i] = B.lp[i] / B.w[i];
        B.lhm[i] = B.lm[i] / B.w[i];
    }
    // strong-form derivative (BR2 lifting): Dstr[i][lam] = l_lam'(xi_i); its interpolant's value at
    // +-1, lDp[lam] = sum_i l_i(+1) Dstr[i][lam] (lDm likewise); the local lifting of one face
    // evaluated on that face, c_+- = sum_i l_i(+-1)^2 / omega_i
    B.Dstr = Dstd;
    B.lDp.assign(NP, 0.0);
    B.lDm.assign(NP, 0.0);
    B.cp = 0.0;
    B.cm = 0.0;
    for (int i = 0; i < NP; ++i) {
        for (int lam = 0; lam < NP; ++lam) {
            B.lDp[lam] += B.lp[i] * Dstd[i * NP + lam];
            B.lDm[lam] += B.lm[i] * Dstd[i * NP + lam];
        }
        B.cp += B.lp[i] * B.lhp[i];
        B.cm += B.lm[i] * B.lhm[i];
    }
    return true;
}
