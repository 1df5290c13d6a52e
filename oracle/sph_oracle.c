/*
 * sph_oracle.c -- the oracle for the SPH neighbour loops.
 *
 * TEST INFRASTRUCTURE ONLY. This file is a plain, slow, obviously correct
 * FP64 CPU implementation of what the density, ghost and force passes
 * compute, written from the definitions in the paper (Schaller et al.,
 * "SWIFT", Section 3). Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it. It shares no code, header or
 * constant with the HIP library, and the library never calls it.
 *
 * Every receiver i is summed over its neighbours j in increasing index
 * order, one pair at a time, with no blocking or reordering. The neighbour
 * set is either every particle (brute force, cand_off == NULL) or an
 * ascending candidate list per receiver (produced by the Python layer from a
 * k-d tree as a superset); in both cases the exact membership test below
 * decides, so both modes give bit-identical results.
 *
 * Readings of the paper taken here (each one also listed in the design notes):
 *  - kernel: Wendland C2 in 3D by default, W(r,h) = 21/(2 pi H^3) (4u^5 -
 *    15u^4 + 20u^3 - 10u^2 + 1), u = r/H, H = gamma_k h (Sections 3.1 and
 *    4.1); gamma_k is a parameter (sqrt(15)/2 for h = twice the kernel's
 *    standard deviation). Section 3.1 also names the Wendland C4 and C6
 *    functions and the cubic, quartic and quintic B-splines; they are
 *    written below in their usual forms on the support [0, H), each scaled
 *    to unit integral over 3D space (the paper asks every kernel to be
 *    normalised), see or_kernel.
 *  - the self term is included in rho, n and their h-derivatives and excluded
 *    from the neighbour count; j is a neighbour of i iff r_ij < H_i (strict).
 *  - velocity divergence and curl use the difference form v_j - v_i in the
 *    paper's smoothed-derivative estimators; the curl is that of the kernel
 *    interpolant, grad W x v (only its magnitude enters the Balsara switch).
 *  - f_i = [1 + h_i/(3 rho_i) d rho_i/dh]^-1 (the inverse is the one written
 *    in the comoving section).
 *  - viscosity: alpha_ij = mean(alpha_V) * mean(B) (the symmetric form of the
 *    default scheme), nu_ij uses the mean density 0.5(rho_i + rho_j), and the
 *    kernel-gradient factor of both the momentum and the energy terms is
 *    G_ij = f_i W'(r,h_i) + f_j W'(r,h_j), which makes the pair exchange
 *    conserve momentum and energy exactly.
 *  - conduction: scalar radial gradient G_ij, v_c uses rho_i + rho_j.
 *  - force neighbours: j != i with r_ij < max(H_i, H_j).
 *  - friends-of-friends (Section 9.1): linked iff the minimum-image squared
 *    distance, formed in FP64 as (dx dx + dy dy) + dz dz, is below b^2; a
 *    group is named by its smallest index.
 *  - short-range gravity (Sections 4.1 and 4.4): the truncated potential is
 *    the product of the softened potential and erfc(r / 2 r_s), the force
 *    its exact gradient; the printed outer force branch r^-3 is read as the
 *    magnitude of -x/r^3.
 *  - SPHENIX viscosity switch (Section 3.3): the printed update is garbled;
 *    it is read as a rise to the target and an exponential decay towards
 *    it. The pins fix this reading's own properties; its agreement with the
 *    printed equation is parity unpinned.
 *  - SPHENIX conduction (Section 3.3): the Laplacian of u, which the paper
 *    names but does not print, is Brookshaw's second-derivative estimator
 *    2 sum (m_j/rho_j)(u_i - u_j) W'/r over r < H_i; the particle's
 *    conduction speed is the largest pair speed v_c,ij over the same
 *    neighbours and alpha_V,max,i the largest alpha_V among them and i; the
 *    conduction parameter's equation, linear with constant coefficients over
 *    a step, is integrated exactly, then capped by the shock limiter.
 *  - time step (Section 3.4): the CFL condition, named but not printed, is
 *    read as dt = c_cfl H / v_sig; the first limiter caps a step at Delta
 *    times the smallest step among the force-loop neighbours.
 *  - Anarchy-PU (Appendix A): the printed conduction speed c_s,i + v_c,j +
 *    mu_ij is read as c_i + c_j + mu_ij (the signal velocity with the sign
 *    of mu reversed, as the text says); the conduction parameter evolves
 *    with beta_c = 0.01 and only the plain cap alpha_c <= 1 (no shock
 *    limiter); the viscosity switch decays with ell = 0.25.
 *  - pressure-energy (Appendix A): the factors f_ij take the form printed
 *    for this flavour, with the number density n = sum_j W_ij in both
 *    brackets (the generic form of Section 3.2 prints the smoothed b there);
 *    du/dt is the energy-conserving partner of the printed acceleration;
 *    the sound speed is sqrt(gamma P_hat / rho); the viscosity is that of
 *    the density flavours and there is no conduction.
 *  - GDF (Appendix A): the mean gradient is G / 2 with G = f_i W'_i + f_j
 *    W'_j (f the geometric-density correction), both terms gradients with
 *    respect to the receiver's position (the printed second term carries
 *    the source's); |S| is the square root of the summed squares of the
 *    trace-free shear (the paper prints the plain sum), the divergence
 *    removed from its diagonal being the trace of the same tensor V; the conduction term is taken with the sign that carries heat
 *    from hot to cold; a receiver without neighbours gets f = 1 and
 *    alpha_c = 0; the viscosity is that of the density flavours and the
 *    alpha_V evolution from the shock detector is not built.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define OR_PI 3.14159265358979323846

/* Wendland C2, 3D (Section 4.1 prints the polynomial; Section 3.1 defines
 * W(r,h) = h^-3 w(r/h) with the cut-off H = gamma_k h). Returns W, dW/dr and
 * dW/dh = -(3/h) W - (r/h) dW/dr (the summand of the paper's dn/dh). */
void or_wc2(double r, double h, double gamma_k, double *w, double *dwdr, double *dwdh)
{
    double H = gamma_k * h;
    double u = r / H;
    if (!(u < 1.0)) {
        *w = 0.0;
        *dwdr = 0.0;
        *dwdh = 0.0;
        return;
    }
    double u2 = u * u, u3 = u2 * u, u4 = u3 * u, u5 = u4 * u;
    double poly = 4.0 * u5 - 15.0 * u4 + 20.0 * u3 - 10.0 * u2 + 1.0;
    double dpoly = 20.0 * u4 - 60.0 * u3 + 60.0 * u2 - 20.0 * u;
    double norm = 21.0 / (2.0 * OR_PI * H * H * H);
    *w = norm * poly;
    *dwdr = norm * dpoly / H;
    *dwdh = -3.0 / h * (*w) - r / h * (*dwdr);
}

void or_wc2_array(int64_t n, const double *r, const double *h, double gamma_k,
                  double *w, double *dwdr, double *dwdh)
{
    for (int64_t k = 0; k < n; ++k)
        or_wc2(r[k], h[k], gamma_k, &w[k], &dwdr[k], &dwdh[k]);
}

/* (x)_+ and its powers, the building block of the B-splines. */
static double pos(double x) { return x > 0.0 ? x : 0.0; }

/* The kernels Section 3.1 lists, as W(r,h) = C H^-3 w(u), u = r/H < 1,
 * H = gamma_k h, with the 3D normalisation C that makes the integral of W
 * over space one. kind: 0 Wendland C2, 1 Wendland C4, 2 Wendland C6 (the
 * Wendland functions psi_{3,k}, k = 1, 2, 3: (1-u)^(2k+2) times their
 * polynomial), 3 cubic, 4 quartic, 5 quintic B-spline (the M4, M5, M6
 * splines as sums of truncated powers (b - u)_+^p with knots spread evenly
 * over the support). w' is the term-by-term derivative of the same
 * expression. Returns W, dW/dr and dW/dh = -(3/h) W - (r/h) dW/dr; 0 for an
 * unknown kind (the callers validate it). */
void or_kernel(int kind, double r, double h, double gamma_k, double *w, double *dwdr,
               double *dwdh)
{
    if (kind == 0) { /* (1-u)^4 (1 + 4u), in the expanded form Section 4.1 prints */
        or_wc2(r, h, gamma_k, w, dwdr, dwdh);
        return;
    }
    double H = gamma_k * h;
    double u = r / H;
    *w = *dwdr = *dwdh = 0.0;
    if (!(u < 1.0))
        return;
    double a = 1.0 - u, C, f, df;
    switch (kind) {
    case 1: /* (1-u)^6 (1 + 6u + 35/3 u^2) */
        C = 495.0 / (32.0 * OR_PI);
        f = pow(a, 6) * (1.0 + 6.0 * u + 35.0 / 3.0 * u * u);
        df = -6.0 * pow(a, 5) * (1.0 + 6.0 * u + 35.0 / 3.0 * u * u) +
             pow(a, 6) * (6.0 + 70.0 / 3.0 * u);
        break;
    case 2: /* (1-u)^8 (1 + 8u + 25u^2 + 32u^3) */
        C = 1365.0 / (64.0 * OR_PI);
        f = pow(a, 8) * (1.0 + 8.0 * u + 25.0 * u * u + 32.0 * u * u * u);
        df = -8.0 * pow(a, 7) * (1.0 + 8.0 * u + 25.0 * u * u + 32.0 * u * u * u) +
             pow(a, 8) * (8.0 + 50.0 * u + 96.0 * u * u);
        break;
    case 3: /* (1-u)^3 - 4 (1/2-u)_+^3 */
        C = 16.0 / OR_PI;
        f = pow(a, 3) - 4.0 * pow(pos(0.5 - u), 3);
        df = -3.0 * pow(a, 2) + 12.0 * pow(pos(0.5 - u), 2);
        break;
    case 4: /* (1-u)^4 - 5 (3/5-u)_+^4 + 10 (1/5-u)_+^4 */
        C = 15625.0 / (512.0 * OR_PI);
        f = pow(a, 4) - 5.0 * pow(pos(0.6 - u), 4) + 10.0 * pow(pos(0.2 - u), 4);
        df = -4.0 * pow(a, 3) + 20.0 * pow(pos(0.6 - u), 3) - 40.0 * pow(pos(0.2 - u), 3);
        break;
    case 5: /* (1-u)^5 - 6 (2/3-u)_+^5 + 15 (1/3-u)_+^5 */
        C = 2187.0 / (40.0 * OR_PI);
        f = pow(a, 5) - 6.0 * pow(pos(2.0 / 3.0 - u), 5) + 15.0 * pow(pos(1.0 / 3.0 - u), 5);
        df = -5.0 * pow(a, 4) + 30.0 * pow(pos(2.0 / 3.0 - u), 4) -
             75.0 * pow(pos(1.0 / 3.0 - u), 4);
        break;
    default:
        return;
    }
    double norm = C / (H * H * H);
    *w = norm * f;
    *dwdr = norm * df / H;
    *dwdh = -3.0 / h * (*w) - r / h * (*dwdr);
}

void or_kernel_array(int kind, int64_t n, const double *r, const double *h, double gamma_k,
                     double *w, double *dwdr, double *dwdh)
{
    for (int64_t k = 0; k < n; ++k)
        or_kernel(kind, r[k], h[k], gamma_k, &w[k], &dwdr[k], &dwdh[k]);
}

/* Minimum-image separation along one axis of a periodic box. */
static double min_image(double d, double L, int periodic)
{
    if (!periodic)
        return d;
    return d - L * nearbyint(d / L);
}

/*
 * Density pass (Section 3.1: number density, its h-derivative, mass density;
 * smoothed divergence and curl of v). For receiver k (particle i = recv[k],
 * or i = k when recv is NULL):
 *   n_i      = sum_j W(r_ij, h_i)                (self included)
 *   dn_i/dh  = sum_j dW/dh(r_ij, h_i)
 *   rho_i    = sum_j m_j W(r_ij, h_i)
 *   drho_i/dh= sum_j m_j dW/dh(r_ij, h_i)
 *   div_sum  = sum_{j!=i} m_j (v_j - v_i) . grad_i W_ij
 *   curl_sum = sum_{j!=i} m_j grad_i W_ij x (v_j - v_i)
 *   nngb_i   = #{ j != i : r_ij < H_i }
 * with grad_i W_ij = dW/dr (r_ij, h_i) x_ij / r_ij and x_ij = x_i - x_j
 * (minimum image). Returns the total neighbour count.
 */
int64_t or_density(int64_t n, const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz,
                   const double *m, const double *h, const double *box, int periodic,
                   double gamma_k, int kernel, int64_t nrecv, const int64_t *recv,
                   const int64_t *cand_off, const int64_t *cand_idx,
                   double *rho, double *rho_dh, double *nd, double *nd_dh,
                   double *div_sum, double *curl_x, double *curl_y, double *curl_z,
                   int64_t *nngb)
{
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t k = 0; k < nrecv; ++k) {
        int64_t i = recv ? recv[k] : k;
        double hi = h[i], Hi = gamma_k * hi;
        double s_rho = 0, s_rho_dh = 0, s_n = 0, s_n_dh = 0;
        double s_div = 0, s_cx = 0, s_cy = 0, s_cz = 0;
        int64_t cnt = 0;
        int64_t jb = cand_off ? cand_off[k] : 0;
        int64_t je = cand_off ? cand_off[k + 1] : n;
        for (int64_t q = jb; q < je; ++q) {
            int64_t j = cand_off ? cand_idx[q] : q;
            double dx = min_image(x[i] - x[j], box[0], periodic);
            double dy = min_image(y[i] - y[j], box[1], periodic);
            double dz = min_image(z[i] - z[j], box[2], periodic);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (!(r < Hi))
                continue;
            double w, dwdr, dwdh;
            or_kernel(kernel, r, hi, gamma_k, &w, &dwdr, &dwdh);
            s_n += w;
            s_n_dh += dwdh;
            s_rho += m[j] * w;
            s_rho_dh += m[j] * dwdh;
            if (j == i)
                continue;
            cnt += 1;
            if (r > 0.0) {
                double gx = dwdr * dx / r, gy = dwdr * dy / r, gz = dwdr * dz / r;
                double wx = vx[j] - vx[i], wy = vy[j] - vy[i], wz = vz[j] - vz[i];
                s_div += m[j] * (wx * gx + wy * gy + wz * gz);
                /* curl of the interpolant: grad W x (v_j - v_i) */
                s_cx += m[j] * (gy * wz - gz * wy);
                s_cy += m[j] * (gz * wx - gx * wz);
                s_cz += m[j] * (gx * wy - gy * wx);
            }
        }
        rho[k] = s_rho;
        rho_dh[k] = s_rho_dh;
        nd[k] = s_n;
        nd_dh[k] = s_n_dh;
        div_sum[k] = s_div;
        curl_x[k] = s_cx;
        curl_y[k] = s_cy;
        curl_z[k] = s_cz;
        nngb[k] = cnt;
        total += cnt;
    }
    return total;
}

/*
 * Smoothed pressure of the pressure-energy flavour (Appendix A, pressure-
 * smoothed SPH) at the receiver's h, over the density neighbours r_ij < H_i
 * with the receiver's own particle included (as for rho):
 *   P_hat_i    = (gamma - 1) sum_j m_j u_j W(r_ij, h_i),
 *   P_hat_dh_i = (gamma - 1) sum_j m_j u_j dW/dh(r_ij, h_i).
 */
void or_pressure(int64_t n, const double *x, const double *y, const double *z,
                 const double *m, const double *u, const double *h, const double *box,
                 int periodic, double gamma_k, int kernel, double gamma_gas, int64_t nrecv,
                 const int64_t *recv, const int64_t *cand_off, const int64_t *cand_idx,
                 double *P_hat, double *P_hat_dh)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrecv; ++k) {
        int64_t i = recv ? recv[k] : k;
        double hi = h[i], Hi = gamma_k * hi;
        double s_p = 0, s_p_dh = 0;
        int64_t jb = cand_off ? cand_off[k] : 0;
        int64_t je = cand_off ? cand_off[k + 1] : n;
        for (int64_t q = jb; q < je; ++q) {
            int64_t j = cand_off ? cand_idx[q] : q;
            double dx = min_image(x[i] - x[j], box[0], periodic);
            double dy = min_image(y[i] - y[j], box[1], periodic);
            double dz = min_image(z[i] - z[j], box[2], periodic);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (!(r < Hi))
                continue;
            double w, dwdr, dwdh;
            or_kernel(kernel, r, hi, gamma_k, &w, &dwdr, &dwdh);
            s_p += m[j] * u[j] * w;
            s_p_dh += m[j] * u[j] * dwdh;
        }
        P_hat[k] = (gamma_gas - 1.0) * s_p;
        P_hat_dh[k] = (gamma_gas - 1.0) * s_p_dh;
    }
}

/*
 * One Newton-Raphson update of h on the partition-of-unity condition
 * (Section 3.1), n(h) (h/eta)^3 = 1, taken in the variable ln h:
 *   G(ln h) = ln(n h^3 / eta^3) = 0,   dG/d ln h = 3 + (h/n) dn/dh,
 *   ln h_new = ln h - G / G'.
 * (The paper names the method and the condition, not the variable; in ln h a
 * uniform medium converges in one step from any start.) The step is limited
 * to a factor 2 either way and to h <= h_max; when G' is not positive the
 * step is a halving or doubling in the direction of -G. The particle is
 * converged when the change is below h_tol * h; its h then stays at the value
 * the sums were evaluated at.
 *
 * Safeguard: h_lo / h_hi carry, per particle, the largest h seen with G < 0
 * and the smallest with G > 0 (0 and +inf before any); the root lies between.
 * Once both are known, a Newton step that would not converge and does not
 * land strictly inside (h_lo, h_hi) is replaced by the geometric midpoint
 * sqrt(h_lo h_hi) (a bisection in ln h), so the iteration cannot cycle where
 * G is nearly flat.
 */
void or_h_update(int64_t n, const double *h, const double *nd, const double *nd_dh,
                 double eta, double h_tol, double h_max, double *h_lo, double *h_hi,
                 double *h_new, int32_t *converged)
{
    const double ln2 = log(2.0);
    for (int64_t k = 0; k < n; ++k) {
        double hk = h[k];
        double G = log(nd[k] * hk * hk * hk / (eta * eta * eta));
        double dG = 3.0 + hk * nd_dh[k] / nd[k];
        if (G < 0.0 && hk > h_lo[k])
            h_lo[k] = hk;
        if (G > 0.0 && hk < h_hi[k])
            h_hi[k] = hk;
        double step;
        if (dG > 0.0 && isfinite(G / dG))
            step = -G / dG;
        else
            step = (G < 0.0) ? ln2 : -ln2;
        if (step > ln2)
            step = ln2;
        if (step < -ln2)
            step = -ln2;
        double hn = hk * exp(step);
        if (hn > h_max)
            hn = h_max;
        if (!(fabs(hn - hk) < h_tol * hk) && h_lo[k] > 0.0 && isfinite(h_hi[k]) &&
            !(hn > h_lo[k] && hn < h_hi[k]))
            hn = sqrt(h_lo[k] * h_hi[k]);
        if (fabs(hn - hk) < h_tol * hk) {
            converged[k] = 1;
            h_new[k] = hk;
        } else {
            converged[k] = 0;
            h_new[k] = hn;
        }
    }
}

/*
 * Ghost (Section 3.1 equation of state; Section 3.2 f-factor and Balsara
 * switch): from the density sums at the final h,
 *   P = (gamma - 1) u rho,  c = sqrt(gamma P / rho),
 *   f = 1 / (1 + h/(3 rho) drho/dh),
 *   div v = div_sum / rho,  |curl v| = |curl_sum| / rho,
 *   B = |div v| / (|div v| + |curl v| + eps c / h),
 *   A = f P / rho^2.
 * With flavour 1 (density-entropy, Section 3.2) the input u is the
 * adiabat A_i and P = A_i rho^gamma; the rest is unchanged.
 * With flavour 3 (pressure-energy, Appendix A; also flavour 4, Anarchy-PU,
 * which is built on it) the pressure is the smoothed
 * one, P = P_hat (or_pressure), c = sqrt(gamma P_hat / rho), and A returns
 * the grad-h term of its factors f_ij = 1 - A_i / (m_j u_j),
 *   A_i = [h_i dP_hat_i/dh / ((gamma - 1) 3 n_i)] / [1 + h_i/(3 n_i) dn_i/dh],
 * with n the number density; f, div, curl and B as for the other flavours
 * (B with this sound speed). nd, nd_dh, P_hat and P_hat_dh are read only
 * for flavours 3 and 4 (NULL otherwise).
 */
void or_ghost(int64_t n, const double *rho, const double *rho_dh, const double *div_sum,
              const double *curl_x, const double *curl_y, const double *curl_z,
              const double *u, const double *h, double gamma_gas, double eps_b,
              double *f, double *P, double *c, double *balsara, double *A,
              double *div_v, double *curl_v, int flavour, const double *nd,
              const double *nd_dh, const double *P_hat, const double *P_hat_dh)
{
    const int entropy = flavour == 1, pe = flavour == 3 || flavour == 4;
    for (int64_t k = 0; k < n; ++k) {
        double r = rho[k];
        /* density-energy: u is the internal energy; density-entropy (the
         * Gadget2 flavour of Section 3.2): u holds the adiabat A, and the
         * equation of state is its other printed form A rho^gamma */
        if (pe)
            P[k] = P_hat[k];
        else
            P[k] = entropy ? u[k] * pow(r, gamma_gas) : (gamma_gas - 1.0) * u[k] * r;
        c[k] = sqrt(gamma_gas * P[k] / r);
        f[k] = 1.0 / (1.0 + h[k] / (3.0 * r) * rho_dh[k]);
        div_v[k] = div_sum[k] / r;
        curl_v[k] = sqrt(curl_x[k] * curl_x[k] + curl_y[k] * curl_y[k] + curl_z[k] * curl_z[k]) / r;
        double ad = fabs(div_v[k]);
        balsara[k] = ad / (ad + curl_v[k] + eps_b * c[k] / h[k]);
        if (pe)
            A[k] = (h[k] * P_hat_dh[k] / ((gamma_gas - 1.0) * 3.0 * nd[k])) /
                   (1.0 + h[k] / (3.0 * nd[k]) * nd_dh[k]);
        else
            A[k] = f[k] * P[k] / (r * r);
    }
}

/*
 * Force pass (Section 3.2 density-energy equations of motion, artificial
 * viscosity with the Balsara switch, Section 3.3 symmetric alpha_ij and the
 * artificial conduction term). For receiver i and every j != i with
 * r_ij < max(H_i, H_j):
 *   g_i = dW/dr(r_ij, h_i), g_j = dW/dr(r_ij, h_j)   (zero outside support)
 *   e = x_ij / r_ij, v_ij = v_i - v_j
 *   mu = min(0, v_ij . x_ij) / r_ij
 *   vsig_ij = c_i + c_j - beta mu
 *   alpha_ij = (alpha_V,i + alpha_V,j)/2 * (B_i + B_j)/2
 *   nu = -alpha_ij mu vsig_ij / (0.5 (rho_i + rho_j))
 *   G = f_i g_i + f_j g_j      (each term only inside its own support)
 *   a_i  -= m_j [A_i g_i + A_j g_j + nu G / 2] e          (A = f P / rho^2)
 *   du_i += m_j [A_i g_i + nu G / 4] (v_ij . e)
 *   du_i += m_j alpha_c,ij v_c,ij (u_i - u_j) G / (rho_i + rho_j)
 *   alpha_c,ij = (P_i alpha_c,i + P_j alpha_c,j) / (P_i + P_j)
 *   v_c,ij = |v_ij . e| + sqrt(2 |P_i - P_j| / (rho_i + rho_j))
 *   vsig_i = max(2 c_i, max_j vsig_ij)
 * Coincident pairs (r = 0) are counted but add nothing (every term carries
 * a kernel gradient, which vanishes at r = 0). Returns the total count.
 * flavour 1 (density-entropy, the Gadget2 flavour of Section 3.2: the input
 * u holds the adiabat A, dA/dt = 0 but for the viscous heating): there is no
 * conduction, du receives dA/dt = (gamma - 1) rho_i^(1 - gamma)
 * sum_j m_j (nu G / 4) (v_ij . e), and du_energy (if not NULL) the
 * internal-energy rate sum_j m_j [A_i g_i + nu G / 4] (v_ij . e).
 * flavour 2 (the Phantom-like flavour of Appendix A): conduction with
 * alpha_c = 1 for every particle and v_c,ij = sqrt(2 |P_i - P_j| / (rho_i +
 * rho_j)); the rest as flavour 0 (density-energy).
 * flavour 3 (pressure-energy, Appendix A): P holds the smoothed pressure
 * P_hat and F the ghost's grad-h terms; with f_ij = 1 - F_i / (m_j u_j),
 * f_ji = 1 - F_j / (m_i u_i) and K_ij = (gamma - 1)^2 u_i u_j,
 *   a_i  -= m_j [K_ij (f_ij g_i / P_i + f_ji g_j / P_j) + nu G / 2] e
 *   du_i += m_j [K_ij f_ij g_i / P_i + nu G / 4] (v_ij . e)
 * (the internal-energy equation is the one that conserves the total energy
 * with this acceleration), the same viscosity as the density flavours (f,
 * rho and c of the ghost) and no conduction. F is read only for flavours 3
 * and 4.
 * flavour 5 (Gasoline-2-like GDF, Appendix A): f holds the GDF correction
 * of or_gdf and alpha_c its conduction parameter; with the mean gradient
 * G / 2,
 *   a_i  -= m_j [(P_i + P_j) G / (2 rho_i rho_j) + nu G / 2] e
 *   du_i += m_j [P_i G / (2 rho_i rho_j) + nu G / 4] (v_ij . e)
 *           + m_j (alpha_c,i + alpha_c,j)(u_i - u_j) G / ((rho_i + rho_j) r)
 * and the density flavours' viscosity (the paper prints no GDF viscosity
 * force; its alpha_V evolution from a shock detector is not built here).
 * flavour 4 (Anarchy-PU, Appendix A): flavour 3 plus conduction with the
 * arithmetic mean alpha_c,ij = (alpha_c,i + alpha_c,j) / 2 and the speed
 * v_c,ij = c_i + c_j + mu (mu <= 0 as in the viscosity):
 *   du_i += m_j alpha_c,ij v_c,ij (u_i - u_j) G / (rho_i + rho_j).
 */
int64_t or_force(int64_t n, const double *x, const double *y, const double *z,
                 const double *vx, const double *vy, const double *vz,
                 const double *m, const double *u, const double *h,
                 const double *rho, const double *P, const double *c, const double *f,
                 const double *balsara, const double *alpha_v, const double *alpha_c,
                 const double *box, int periodic, double gamma_k, int kernel, double beta_v,
                 int64_t nrecv, const int64_t *recv,
                 const int64_t *cand_off, const int64_t *cand_idx,
                 double *ax, double *ay, double *az, double *du, double *vsig, int64_t *nforce,
                 int flavour, double gamma_gas, double *du_energy, const double *F)
{
    const int entropy = flavour == 1, phantom = flavour == 2;
    const int pe = flavour == 3 || flavour == 4, anarchy = flavour == 4;
    const int gdf = flavour == 5;
    const double gm1sq = (gamma_gas - 1.0) * (gamma_gas - 1.0);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t k = 0; k < nrecv; ++k) {
        int64_t i = recv ? recv[k] : k;
        double Hi = gamma_k * h[i];
        double Ai = pe ? 0.0 : f[i] * P[i] / (rho[i] * rho[i]);
        double s_ax = 0, s_ay = 0, s_az = 0, s_du = 0, s_visc = 0;
        double s_vsig = 2.0 * c[i];
        int64_t cnt = 0;
        int64_t jb = cand_off ? cand_off[k] : 0;
        int64_t je = cand_off ? cand_off[k + 1] : n;
        for (int64_t q = jb; q < je; ++q) {
            int64_t j = cand_off ? cand_idx[q] : q;
            if (j == i)
                continue;
            double Hj = gamma_k * h[j];
            double dx = min_image(x[i] - x[j], box[0], periodic);
            double dy = min_image(y[i] - y[j], box[1], periodic);
            double dz = min_image(z[i] - z[j], box[2], periodic);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double Hmax = Hi > Hj ? Hi : Hj;
            if (!(r < Hmax))
                continue;
            cnt += 1;
            if (!(r > 0.0))
                continue;
            double w, gi, gj, dwdh;
            or_kernel(kernel, r, h[i], gamma_k, &w, &gi, &dwdh);
            or_kernel(kernel, r, h[j], gamma_k, &w, &gj, &dwdh);
            double ex = dx / r, ey = dy / r, ez = dz / r;
            double wx = vx[i] - vx[j], wy = vy[i] - vy[j], wz = vz[i] - vz[j];
            double vdotx = wx * dx + wy * dy + wz * dz;
            double vdote = wx * ex + wy * ey + wz * ez;
            double mu = vdotx < 0.0 ? vdotx / r : 0.0;
            double vsig_ij = c[i] + c[j] - beta_v * mu;
            double alpha_ij = 0.5 * (alpha_v[i] + alpha_v[j]) * 0.5 * (balsara[i] + balsara[j]);
            double nu = -alpha_ij * mu * vsig_ij / (0.5 * (rho[i] + rho[j]));
            double Aj = pe ? 0.0 : f[j] * P[j] / (rho[j] * rho[j]);
            /* a kernel term outside its own support is zero (W' = 0 there),
             * also when the particle's f is infinite (alone in its support) */
            double fgi = r < Hi ? f[i] * gi : 0.0, Agi = r < Hi ? Ai * gi : 0.0;
            double fgj = r < Hj ? f[j] * gj : 0.0, Agj = r < Hj ? Aj * gj : 0.0;
            if (pe) {
                /* pressure-energy: the pressure terms with the smoothed
                 * pressure and the factors f_ij, f_ji */
                double K = gm1sq * u[i] * u[j];
                double fij = 1.0 - F[i] / (m[j] * u[j]);
                double fji = 1.0 - F[j] / (m[i] * u[i]);
                Agi = r < Hi ? K * fij * gi / P[i] : 0.0;
                Agj = r < Hj ? K * fji * gj / P[j] : 0.0;
            }
            double G = fgi + fgj;
            if (gdf) {
                /* GDF (Appendix A): both pressures over rho_i rho_j on the
                 * mean gradient G / 2 (f the GDF correction); du/dt takes
                 * the receiver's pressure alone */
                double pij = 0.5 * G / (rho[i] * rho[j]);
                Agi = P[i] * pij;
                Agj = P[j] * pij;
            }
            double acc = Agi + Agj + 0.5 * nu * G;
            s_ax -= m[j] * acc * ex;
            s_ay -= m[j] * acc * ey;
            s_az -= m[j] * acc * ez;
            s_du += m[j] * (Agi + 0.25 * nu * G) * vdote;
            s_visc += m[j] * 0.25 * nu * G * vdote;
            if (gdf) {
                /* GDF conduction (Appendix A): alpha_c dimensional, the pair
                 * term (alpha_c,i + alpha_c,j)(u_i - u_j)(x_ij . mean
                 * gradient) / (0.5 (rho_i + rho_j) r^2), x_ij . mean gradient
                 * = r G / 2; taken with the sign that carries heat from the
                 * hotter particle to the colder (G < 0) */
                s_du += m[j] * (alpha_c[i] + alpha_c[j]) * (u[i] - u[j]) * G /
                        ((rho[i] + rho[j]) * r);
            } else if (anarchy) {
                /* Anarchy-PU (Appendix A): mean alpha_c and the signal speed
                 * with the sign of mu reversed (and no beta) */
                double v_c = c[i] + c[j] + mu;
                double alpha_c_ij = 0.5 * (alpha_c[i] + alpha_c[j]);
                s_du += m[j] * alpha_c_ij * v_c * (u[i] - u[j]) * G / (rho[i] + rho[j]);
            } else if (phantom) {
                /* Phantom-like (Appendix A): alpha_c = 1 for every particle and
                 * the conduction speed without the velocity term */
                double v_c = sqrt(2.0 * fabs(P[i] - P[j]) / (rho[i] + rho[j]));
                s_du += m[j] * v_c * (u[i] - u[j]) * G / (rho[i] + rho[j]);
            } else if (!entropy && !pe) {
                double psum = P[i] + P[j];
                double alpha_c_ij =
                    psum > 0.0 ? (P[i] * alpha_c[i] + P[j] * alpha_c[j]) / psum : 0.0;
                double v_c = fabs(vdote) + sqrt(2.0 * fabs(P[i] - P[j]) / (rho[i] + rho[j]));
                s_du += m[j] * alpha_c_ij * v_c * (u[i] - u[j]) * G / (rho[i] + rho[j]);
            }
            if (vsig_ij > s_vsig)
                s_vsig = vsig_ij;
        }
        ax[k] = s_ax;
        ay[k] = s_ay;
        az[k] = s_az;
        /* density-entropy: the adiabat changes only by the viscous heating,
         * dA/dt = (gamma - 1) rho^(1 - gamma) du/dt|visc; du_energy keeps the
         * internal-energy rate the forces imply (for the energy balance) */
        du[k] = entropy ? (gamma_gas - 1.0) * pow(rho[i], 1.0 - gamma_gas) * s_visc : s_du;
        if (du_energy)
            du_energy[k] = s_du;
        vsig[k] = s_vsig;
        nforce[k] = cnt;
        total += cnt;
    }
    return total;
}

/* Global conservation sums (the end-of-step reduction of Section 2):
 * out[0..2] = sum m a, out[3] = sum m (v.a + du/dt),
 * out[4] = sum m |a|, out[5] = sum m |du/dt|. Plain sequential FP64 sums. */
void or_sums(int64_t n, const double *m, const double *vx, const double *vy, const double *vz,
             const double *ax, const double *ay, const double *az, const double *du,
             double *out)
{
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = 0; k < n; ++k) {
        s[0] += m[k] * ax[k];
        s[1] += m[k] * ay[k];
        s[2] += m[k] * az[k];
        s[3] += m[k] * (vx[k] * ax[k] + vy[k] * ay[k] + vz[k] * az[k] + du[k]);
        s[4] += m[k] * sqrt(ax[k] * ax[k] + ay[k] * ay[k] + az[k] * az[k]);
        s[5] += m[k] * fabs(du[k]);
    }
    for (int q = 0; q < 6; ++q)
        out[q] = s[q];
}

/*
 * Friends-of-friends groups (Section 9.1): particles i and j are linked when
 * they lie closer than the linking length b, read here as
 * |x_i - x_j|^2 < b^2 for the minimum-image separation, the squared distance
 * formed in FP64 as ((dx dx + dy dy) + dz dz) and compared with b2 = b^2.
 * Groups are the connected components of the links. Plain sequential
 * union-find over the candidate pairs (every pair, or an ascending candidate
 * list per particle), each union hanging the larger root under the smaller,
 * so the root of every set is its smallest index; on return group[i] is the
 * smallest index of i's group. Returns the number of links (pairs i < j).
 */
static int64_t or_find(int64_t *parent, int64_t i)
{
    while (parent[i] != i)
        i = parent[i];
    return i;
}

int64_t or_fof(int64_t n, const double *x, const double *y, const double *z, const double *box,
               int periodic, double b2, const int64_t *cand_off, const int64_t *cand_idx,
               int64_t *group)
{
    for (int64_t i = 0; i < n; ++i)
        group[i] = i;
    int64_t links = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t jb = cand_off ? cand_off[i] : 0;
        int64_t je = cand_off ? cand_off[i + 1] : n;
        for (int64_t q = jb; q < je; ++q) {
            int64_t j = cand_off ? cand_idx[q] : q;
            if (j <= i)
                continue;
            double dx = min_image(x[i] - x[j], box[0], periodic);
            double dy = min_image(y[i] - y[j], box[1], periodic);
            double dz = min_image(z[i] - z[j], box[2], periodic);
            double r2 = dx * dx + dy * dy + dz * dz;
            if (!(r2 < b2))
                continue;
            links += 1;
            int64_t ri = or_find(group, i), rj = or_find(group, j);
            if (ri < rj)
                group[rj] = ri;
            else if (rj < ri)
                group[ri] = rj;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        group[i] = or_find(group, i);
    return links;
}

/*
 * Short-range softened gravity by direct summation (Section 4.1: the C2
 * softened potential; Section 4.4: the short-range truncation of the mesh
 * split). For a pair at separation r:
 *   phi(r)   = f(r/H) / H for r < H, 1/r beyond, with the printed
 *              f(u) = -3u^7 + 15u^6 - 28u^5 + 21u^4 - 7u^2 + 3;
 *   phi'(r)/r = g(r/H) / H^3 for r < H, -1/r^3 beyond, with the printed
 *              g(u) = f'(u)/u = -21u^5 + 90u^4 - 140u^3 + 84u^2 - 14
 *              (the printed outer branch, r^-3, is the magnitude: the
 *              gradient of 1/r is -r/r^3);
 *   chi(r)   = erfc(r / (2 r_s)) (chi = 1 when r_s <= 0: no truncation),
 *   the short-range potential phi_s = phi chi, and the acceleration is its
 *   exact gradient:
 *   a_i      = G sum_j m_j x_ij [phi'(r) chi(r) + phi(r) chi'(r)] / r,
 *   pot_i    = -G sum_j m_j phi(r) chi(r),
 * over j != i with r_ij < r_p2p (the pairs a tree code sums directly), x_ij
 * = x_i - x_j minimum image, chi'(r) = -exp(-r^2 / (4 r_s^2)) / (sqrt(pi)
 * r_s). A coincident pair (r = 0) adds to the potential, not to the force.
 * scale_i = G sum_j m_j |[...] / r| r, the size of the summed terms (the
 * natural scale of the rounding error of the sum). Returns the pair count.
 */
static void or_grav_f_g(double u, double *f, double *g)
{
    double u2 = u * u, u3 = u2 * u, u4 = u3 * u, u5 = u4 * u, u6 = u5 * u, u7 = u6 * u;
    *f = -3.0 * u7 + 15.0 * u6 - 28.0 * u5 + 21.0 * u4 - 7.0 * u2 + 3.0;
    *g = -21.0 * u5 + 90.0 * u4 - 140.0 * u3 + 84.0 * u2 - 14.0;
}

void or_grav_pair(double r, double H, double rs, double *phi_s, double *k_over_r)
{
    double phi, dphi_r; /* phi and phi'(r)/r */
    if (r < H) {
        double f, g;
        or_grav_f_g(r / H, &f, &g);
        phi = f / H;
        dphi_r = g / (H * H * H);
    } else {
        phi = 1.0 / r;
        dphi_r = -1.0 / (r * r * r);
    }
    double chi = 1.0, dchi_r = 0.0; /* chi and chi'(r)/r */
    if (rs > 0.0) {
        chi = erfc(r / (2.0 * rs));
        dchi_r = r > 0.0 ? -exp(-r * r / (4.0 * rs * rs)) / (sqrt(OR_PI) * rs) / r : 0.0;
    }
    *phi_s = phi * chi;
    *k_over_r = r > 0.0 ? dphi_r * chi + phi * dchi_r : 0.0;
}

void or_grav_pair_array(int64_t n, const double *r, double H, double rs, double *phi_s,
                        double *k_over_r)
{
    for (int64_t k = 0; k < n; ++k)
        or_grav_pair(r[k], H, rs, &phi_s[k], &k_over_r[k]);
}

int64_t or_gravity(int64_t n, const double *x, const double *y, const double *z, const double *m,
                   const double *box, int periodic, double G, double H, double rs, double rp2p,
                   int64_t nrecv, const int64_t *recv, const int64_t *cand_off,
                   const int64_t *cand_idx, double *ax, double *ay, double *az, double *pot,
                   double *scale)
{
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t k = 0; k < nrecv; ++k) {
        int64_t i = recv ? recv[k] : k;
        double sx = 0, sy = 0, sz = 0, sp = 0, sa = 0;
        int64_t jb = cand_off ? cand_off[k] : 0;
        int64_t je = cand_off ? cand_off[k + 1] : n;
        for (int64_t q = jb; q < je; ++q) {
            int64_t j = cand_off ? cand_idx[q] : q;
            if (j == i)
                continue;
            double dx = min_image(x[i] - x[j], box[0], periodic);
            double dy = min_image(y[i] - y[j], box[1], periodic);
            double dz = min_image(z[i] - z[j], box[2], periodic);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (!(r < rp2p))
                continue;
            total += 1;
            double phi_s, kr;
            or_grav_pair(r, H, rs, &phi_s, &kr);
            sp += m[j] * phi_s;
            sx += m[j] * kr * dx;
            sy += m[j] * kr * dy;
            sz += m[j] * kr * dz;
            sa += m[j] * fabs(kr) * r;
        }
        ax[k] = G * sx;
        ay[k] = G * sy;
        az[k] = G * sz;
        pot[k] = -G * sp;
        scale[k] = G * sa;
    }
    return total;
}

/*
 * SPHENIX viscosity switch (Section 3.3): the time derivative of the
 * velocity divergence from the values at the start and end of the step,
 *   Ddiv = (div_new - div_old) / dt,
 * the shock indicator S = H^2 max(0, -Ddiv) with H = gamma_k h, the local
 * target alpha_loc = alpha_max S / (v_sig^2 + S) (0 where S = 0), then
 *   alpha_new = alpha_loc                                   if alpha_loc > alpha,
 *   alpha_new = alpha_loc + (alpha - alpha_loc) exp(-ell c dt / H)   otherwise:
 * an immediate rise at a shock and an exponential decay towards alpha_loc
 * on the time scale H / (ell c) (the reading of the printed update, which
 * as typeset would lower alpha the more the larger alpha_loc is).
 * alpha is updated in place.
 */
void or_alpha_v_update(int64_t n, const double *div_old, const double *div_new, const double *c,
                       const double *h, const double *vsig, double dt, double gamma_k,
                       double alpha_max, double ell, double *alpha)
{
    for (int64_t i = 0; i < n; ++i) {
        double H = gamma_k * h[i];
        double ddiv = (div_new[i] - div_old[i]) / dt;
        double S = H * H * (ddiv < 0.0 ? -ddiv : 0.0);
        double loc = S > 0.0 ? alpha_max * S / (vsig[i] * vsig[i] + S) : 0.0;
        if (loc > alpha[i])
            alpha[i] = loc;
        else
            alpha[i] = loc + (alpha[i] - loc) * exp(-ell * c[i] * dt / H);
    }
}

/*
 * SPHENIX gradient loop (Section 3.3: the conduction parameter is driven by
 * the Laplacian of the internal energy and decays on the conduction speed;
 * the conduction limiter reads the largest viscosity parameter nearby). For
 * receiver k (particle i) over every j != i with 0 < r_ij < H_i:
 *   lap_u_i  = 2 sum_j (m_j / rho_j) (u_i - u_j) dW/dr(r_ij, h_i) / r_ij
 *              (the paper does not print the estimator; this is the
 *              second-derivative form of Brookshaw, which returns 2 for
 *              u = x^2 in the continuum limit)
 *   vc_i     = max_j [ |v_ij . x_ij| / r_ij + sqrt(2 |P_i - P_j| / (rho_i + rho_j)) ]
 *              (the pair conduction speed of Section 3.3; 0 without neighbours;
 *              with c != NULL, Anarchy-PU of Appendix A, the pair speed is
 *              c_i + c_j + min(0, v_ij . x_ij) / r_ij)
 *   avmax_i  = max(alpha_V,i, max_j alpha_V,j)
 * Coincident pairs (r = 0) have no direction and are skipped. Returns the
 * number of pairs used.
 */
int64_t or_gradient(int64_t n, const double *x, const double *y, const double *z,
                    const double *vx, const double *vy, const double *vz, const double *m,
                    const double *u, const double *h, const double *rho, const double *P,
                    const double *alpha_v, const double *box, int periodic, double gamma_k,
                    int kernel, int64_t nrecv, const int64_t *recv, const int64_t *cand_off,
                    const int64_t *cand_idx, double *lap_u, double *vc, double *avmax,
                    const double *c)
{
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t k = 0; k < nrecv; ++k) {
        int64_t i = recv ? recv[k] : k;
        double hi = h[i], Hi = gamma_k * hi;
        double s_lap = 0.0, s_vc = 0.0, s_av = alpha_v[i];
        int64_t cnt = 0;
        int64_t jb = cand_off ? cand_off[k] : 0;
        int64_t je = cand_off ? cand_off[k + 1] : n;
        for (int64_t q = jb; q < je; ++q) {
            int64_t j = cand_off ? cand_idx[q] : q;
            if (j == i)
                continue;
            double dx = min_image(x[i] - x[j], box[0], periodic);
            double dy = min_image(y[i] - y[j], box[1], periodic);
            double dz = min_image(z[i] - z[j], box[2], periodic);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (!(r < Hi) || !(r > 0.0))
                continue;
            double w, dwdr, dwdh;
            or_kernel(kernel, r, hi, gamma_k, &w, &dwdr, &dwdh);
            s_lap += m[j] / rho[j] * (u[i] - u[j]) * dwdr / r;
            double vdotx = (vx[i] - vx[j]) * dx + (vy[i] - vy[j]) * dy + (vz[i] - vz[j]) * dz;
            double v_c = c ? c[i] + c[j] + (vdotx < 0.0 ? vdotx / r : 0.0)
                           : fabs(vdotx) / r + sqrt(2.0 * fabs(P[i] - P[j]) / (rho[i] + rho[j]));
            if (v_c > s_vc)
                s_vc = v_c;
            if (alpha_v[j] > s_av)
                s_av = alpha_v[j];
            cnt += 1;
        }
        lap_u[k] = 2.0 * s_lap;
        vc[k] = s_vc;
        avmax[k] = s_av;
        total += cnt;
    }
    return total;
}

/*
 * Gasoline-2-like (GDF) flavour, Appendix A: the geometric density average
 * correction f_i and the conduction parameter alpha_c,i from the trace-free
 * shear tensor. For receiver k (particle i) over every j with r_ij < H_i
 * (W_ij = W(r_ij, h_i); the receiver itself adds nothing: r = 0):
 *   S1 = sum_j m_j r_ij^2 W_ij,  S2 = sum_j (m_j / rho_j) r_ij^2 W_ij,
 *   V_ab = sum_j (v_a,i - v_a,j)(x_b,i - x_b,j) m_j W_ij / (S1 / 3),
 *   f_i = (S1 / rho_i) / S2,
 *   S_ab = (V_ab + V_ba) / 2 - delta_ab (V_xx + V_yy + V_zz) / 3,
 *   alpha_c,i = C |S| h_i^2 with |S| = sqrt(sum_ab S_ab^2)
 * (the paper prints |S| as the plain sum of squares; its square root is the
 * reading that gives alpha_c the dimension of a diffusivity, which the
 * conduction term of the energy equation requires). A receiver without a
 * neighbour at r > 0 gets f = 1 and alpha_c = 0.
 */
void or_gdf(int64_t n, const double *x, const double *y, const double *z,
            const double *vx, const double *vy, const double *vz, const double *m,
            const double *h, const double *rho, const double *box, int periodic,
            double gamma_k, int kernel, double C, int64_t nrecv, const int64_t *recv,
            const int64_t *cand_off, const int64_t *cand_idx, double *f_out,
            double *alpha_c_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrecv; ++k) {
        int64_t i = recv ? recv[k] : k;
        double Hi = gamma_k * h[i];
        double S1 = 0.0, S2 = 0.0;
        double V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        int64_t jb = cand_off ? cand_off[k] : 0;
        int64_t je = cand_off ? cand_off[k + 1] : n;
        for (int64_t q = jb; q < je; ++q) {
            int64_t j = cand_off ? cand_idx[q] : q;
            double d[3] = {min_image(x[i] - x[j], box[0], periodic),
                           min_image(y[i] - y[j], box[1], periodic),
                           min_image(z[i] - z[j], box[2], periodic)};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double r = sqrt(r2);
            if (!(r < Hi))
                continue;
            double w, dwdr, dwdh;
            or_kernel(kernel, r, h[i], gamma_k, &w, &dwdr, &dwdh);
            double dv[3] = {vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j]};
            S1 += m[j] * r2 * w;
            S2 += m[j] / rho[j] * r2 * w;
            for (int a2 = 0; a2 < 3; ++a2)
                for (int b2 = 0; b2 < 3; ++b2)
                    V[a2][b2] += dv[a2] * d[b2] * m[j] * w;
        }
        if (!(S1 > 0.0) || !(S2 > 0.0)) {
            f_out[k] = 1.0;
            alpha_c_out[k] = 0.0;
            continue;
        }
        for (int a2 = 0; a2 < 3; ++a2)
            for (int b2 = 0; b2 < 3; ++b2)
                V[a2][b2] /= S1 / 3.0;
        double tr = V[0][0] + V[1][1] + V[2][2];
        double s2 = 0.0;
        for (int a2 = 0; a2 < 3; ++a2)
            for (int b2 = 0; b2 < 3; ++b2) {
                double sab = 0.5 * (V[a2][b2] + V[b2][a2]) - (a2 == b2 ? tr / 3.0 : 0.0);
                s2 += sab * sab;
            }
        f_out[k] = (S1 / rho[i]) / S2;
        alpha_c_out[k] = C * sqrt(s2) * h[i] * h[i];
    }
}

/*
 * GDF shock detector (Appendix A). For receiver k (particle i) over every j
 * with r_ij < H_i (W_ij = W(r_ij, h_i)):
 *   grad P_i = (gamma - 1) sum_j m_j u_j (dW/dr)(r_ij, h_i) x_ij / r_ij
 *              (x_ij = x_i - x_j; pairs at r = 0 have no direction),
 *   n_i = grad P_i / |grad P_i|,  dv/dn_i = sum_ab n_a V_ab n_b with V the
 *   velocity-gradient tensor of or_gdf, div v_i = V_xx + V_yy + V_zz,
 *   D_i = 3/2 [dv/dn_i + max(-div v_i / 3, 0)].
 * A receiver without a pressure gradient (|grad P| = 0) has no direction:
 * dv/dn = 0 there; one without neighbours at r > 0 gets D = 0.
 */
void or_gdf_detector(int64_t n, const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz, const double *m,
                     const double *u, const double *h, const double *box, int periodic,
                     double gamma_k, int kernel, double gamma_gas, int64_t nrecv,
                     const int64_t *recv, const int64_t *cand_off, const int64_t *cand_idx,
                     double *D_out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nrecv; ++k) {
        int64_t i = recv ? recv[k] : k;
        double Hi = gamma_k * h[i];
        double S1 = 0.0, gp[3] = {0, 0, 0};
        double V[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        int64_t jb = cand_off ? cand_off[k] : 0;
        int64_t je = cand_off ? cand_off[k + 1] : n;
        for (int64_t q = jb; q < je; ++q) {
            int64_t j = cand_off ? cand_idx[q] : q;
            double d[3] = {min_image(x[i] - x[j], box[0], periodic),
                           min_image(y[i] - y[j], box[1], periodic),
                           min_image(z[i] - z[j], box[2], periodic)};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double r = sqrt(r2);
            if (!(r < Hi) || !(r > 0.0))
                continue;
            double w, dwdr, dwdh;
            or_kernel(kernel, r, h[i], gamma_k, &w, &dwdr, &dwdh);
            double dv[3] = {vx[i] - vx[j], vy[i] - vy[j], vz[i] - vz[j]};
            S1 += m[j] * r2 * w;
            for (int a2 = 0; a2 < 3; ++a2) {
                gp[a2] += (gamma_gas - 1.0) * m[j] * u[j] * dwdr * d[a2] / r;
                for (int b2 = 0; b2 < 3; ++b2)
                    V[a2][b2] += dv[a2] * d[b2] * m[j] * w;
            }
        }
        if (!(S1 > 0.0)) {
            D_out[k] = 0.0;
            continue;
        }
        for (int a2 = 0; a2 < 3; ++a2)
            for (int b2 = 0; b2 < 3; ++b2)
                V[a2][b2] /= S1 / 3.0;
        double gn = sqrt(gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2]);
        double dvdn = 0.0;
        if (gn > 0.0)
            for (int a2 = 0; a2 < 3; ++a2)
                for (int b2 = 0; b2 < 3; ++b2)
                    dvdn += gp[a2] / gn * V[a2][b2] * gp[b2] / gn;
        double div = V[0][0] + V[1][1] + V[2][2];
        double comp = -div / 3.0;
        D_out[k] = 1.5 * (dvdn + (comp > 0.0 ? comp : 0.0));
    }
}

/*
 * GDF viscosity parameter over a step dt (Appendix A): with dD/dt read as
 * (D_new - D_old) / dt,
 *   A_i = 2 h_i^2 B_i max(-dD/dt, 0),  alpha_loc = alpha_max A_i / (A_i + v_sig,i^2),
 * and, as the paper evolves it like the SPHENIX switch, alpha rises to
 * alpha_loc at once when alpha_loc is larger and otherwise relaxes by
 * d alpha / dt = 0.2 c_i (alpha_loc - alpha) / h_i, linear with constant
 * coefficients over the step, integrated exactly:
 *   alpha = alpha_loc + (alpha - alpha_loc) exp(-0.2 c_i dt / h_i).
 * alpha is updated in place.
 */
void or_gdf_alpha_v_update(int64_t n, const double *D_old, const double *D_new,
                           const double *c, const double *h, const double *vsig,
                           const double *B, double dt, double alpha_max, double *alpha)
{
    for (int64_t i = 0; i < n; ++i) {
        double dD = (D_new[i] - D_old[i]) / dt;
        double A = 2.0 * h[i] * h[i] * B[i] * (dD < 0.0 ? -dD : 0.0);
        double loc = A > 0.0 ? alpha_max * A / (A + vsig[i] * vsig[i]) : 0.0;
        if (loc > alpha[i])
            alpha[i] = loc;
        else
            alpha[i] = loc + (alpha[i] - loc) * exp(-0.2 * c[i] * dt / h[i]);
    }
}

/*
 * SPHENIX conduction parameter over a step dt (Section 3.3): the evolution
 * equation
 *   d alpha_c / dt = beta_c H lap_u / sqrt(u) - (alpha_c - alpha_c,min) vc / H
 * has constant coefficients over the step, so it is integrated exactly: with
 * S = beta_c H lap_u / sqrt(u) and lam = vc / H,
 *   alpha = a_inf + (alpha - a_inf) exp(-lam dt),  a_inf = alpha_c,min + S / lam,
 * and alpha + S dt where lam = 0 (its limit). Then the shock limiter caps
 * it at alpha_c,max (1 - avmax / alpha_V,max) and it is kept >= alpha_c,min
 * (beta_c = 1, alpha_c,min = 0, alpha_c,max = 1, alpha_V,max = 2 as
 * printed). alpha is updated in place.
 */
void or_alpha_c_update(int64_t n, const double *lap_u, const double *u, const double *h,
                       const double *vc, const double *avmax, double dt, double gamma_k,
                       double beta_c, double a_min, double a_max, double av_max, double *alpha)
{
    for (int64_t i = 0; i < n; ++i) {
        double H = gamma_k * h[i];
        double S = u[i] > 0.0 ? beta_c * H * lap_u[i] / sqrt(u[i]) : 0.0;
        double lam = vc[i] / H;
        double a = alpha[i];
        if (lam > 0.0) {
            double a_inf = a_min + S / lam;
            a = a_inf + (a - a_inf) * exp(-lam * dt);
        } else {
            a = a + S * dt;
        }
        double cap = a_max * (1.0 - avmax[i] / av_max);
        if (cap < a_min)
            cap = a_min;
        if (a > cap)
            a = cap;
        if (a < a_min)
            a = a_min;
        alpha[i] = a;
    }
}

/*
 * Time-step size (Section 3.4: the CFL condition, then the first limiter).
 * The paper names the condition without printing it; here the Courant form
 * on the kernel support, dt_i = c_cfl H_i / v_sig,i. The limiter: no
 * particle's step exceeds delta times the smallest step among the particles
 * it interacts with in the force loop (j != i, r_ij < max(H_i, H_j)):
 *   dt_out_i = min(dt_i, delta min_j dt_j).
 * or_dt_cfl fills dt from h and v_sig; or_dt_limit applies the limiter for
 * the receivers (cand lists as in the force pass) and returns the pair count.
 */
void or_dt_cfl(int64_t n, const double *h, const double *vsig, double gamma_k, double c_cfl,
               double *dt)
{
    for (int64_t i = 0; i < n; ++i)
        dt[i] = c_cfl * gamma_k * h[i] / vsig[i];
}

int64_t or_dt_limit(int64_t n, const double *x, const double *y, const double *z,
                    const double *h, const double *dt, const double *box, int periodic,
                    double gamma_k, double delta, int64_t nrecv, const int64_t *recv,
                    const int64_t *cand_off, const int64_t *cand_idx, double *dt_out)
{
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t k = 0; k < nrecv; ++k) {
        int64_t i = recv ? recv[k] : k;
        double Hi = gamma_k * h[i];
        double lim = dt[i];
        int64_t jb = cand_off ? cand_off[k] : 0;
        int64_t je = cand_off ? cand_off[k + 1] : n;
        for (int64_t q = jb; q < je; ++q) {
            int64_t j = cand_off ? cand_idx[q] : q;
            if (j == i)
                continue;
            double dx = min_image(x[i] - x[j], box[0], periodic);
            double dy = min_image(y[i] - y[j], box[1], periodic);
            double dz = min_image(z[i] - z[j], box[2], periodic);
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double Hj = gamma_k * h[j];
            if (!(r < (Hi > Hj ? Hi : Hj)))
                continue;
            total += 1;
            if (delta * dt[j] < lim)
                lim = delta * dt[j];
        }
        dt_out[k] = lim;
    }
    return total;
}

/*
 * Leapfrog operators (Section 2.4: kick-drift-kick). A half kick adds
 * a dt/2 to v and du/dt dt/2 to u; a drift moves x by v dt, wrapped into
 * [0, L) in a periodic box.
 */
void or_kick(int64_t n, double *vx, double *vy, double *vz, double *u, const double *ax,
             const double *ay, const double *az, const double *du, double dt_half)
{
    for (int64_t i = 0; i < n; ++i) {
        vx[i] += ax[i] * dt_half;
        vy[i] += ay[i] * dt_half;
        vz[i] += az[i] * dt_half;
        u[i] += du[i] * dt_half;
    }
}

void or_drift(int64_t n, double *x, double *y, double *z, const double *vx, const double *vy,
              const double *vz, double dt, const double *box, int periodic)
{
    for (int64_t i = 0; i < n; ++i) {
        double p[3] = {x[i] + vx[i] * dt, y[i] + vy[i] * dt, z[i] + vz[i] * dt};
        for (int a = 0; a < 3; ++a)
            if (periodic) {
                p[a] -= box[a] * floor(p[a] / box[a]);
                if (p[a] >= box[a])  /* a tiny negative p rounds up to L */
                    p[a] -= box[a];
            }
        x[i] = p[0];
        y[i] = p[1];
        z[i] = p[2];
    }
}
