/*
 * fft_oracle.c -- plain FP64 CPU oracle for the spectral PDE solvers.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this.  It shares no code, header,
 * table or helper with the GPU library; the two are compared, never mixed.
 *
 * Everything is written for a reader holding the paper (arXiv 2412.12308):
 *
 *   - 1D transform: recursive radix-2 decimation in time (Sec. II.C, the
 *     even/odd split and the butterfly pair Eq. (FFTpairodd) and
 *     Eq. (FFTpairodd_2)), recursing down to length 1.  Twiddles
 *     w^k = exp(sign * 2 pi i k / N) come straight from libm cos/sin.
 *   - Lengths that are not powers of two (Sec. II.D restricts the method to
 *     N = 2^m; other lengths are an extension): the sum of Eq. (DFT)
 *     evaluated term by term, O(N^2) per line, with the product j k reduced
 *     modulo N in integers before the angle 2 pi (j k mod N)/N is formed.
 *   - Sign convention: the forward transform uses exp(-2 pi i ...), the sign
 *     of the row-column derivation in Sec. II.D; the inverse uses
 *     exp(+2 pi i ...) and the 1/N factor of the iDFT in Sec. II.B.  (The
 *     paper's Eq. (DFT) writes omega_N = exp(+2 pi i/N); the two readings
 *     differ only by the index reversal P_k <-> P_{-k}, and every solver
 *     below is insensitive to it because its symbol is even in k.)
 *   - 2D transform: all rows (x direction, fixed y index) first, then all
 *     columns (y direction, fixed x frequency), Sec. II.D.
 *   - Poisson (Sec. III.A): u = F^-1{ -F{g} / |k|^2 }, g = s - mean(s), i.e.
 *     the k = 0 coefficient of the right-hand side is dropped and the k = 0
 *     coefficient of u is set to 0 (zero-mean solution), Eq. (Poisson2),
 *     Eq. (SolutionPoisson).
 *   - Diffusion (Sec. III.B, source-free): u^(t) = f^ exp(-kappa |k|^2 t),
 *     Eq. (solCalorFourier) with a diffusivity kappa.
 *   - Wave (Sec. III.C, s = 0): u^(t) = f^ cos(w t) + g^ sin(w t)/w for
 *     w = c|k| != 0 and f^ + g^ t for w = 0, Eq. (OmegaNonZero) and
 *     Eq. (OmegaZero); the velocity is its time derivative,
 *     v^(t) = -w f^ sin(w t) + g^ cos(w t).
 *   - Sources constant in time (Sec. III.B, III.C): forced decay and the
 *     forced oscillator per coefficient, with the constant particular
 *     solution of the oscillator written out (see oracle_solve_wave_source).
 *   - Wavenumbers: angular k = 2 pi a'/L with a' the signed index
 *     (a' = a for a < N/2, a - N otherwise), Sec. II.D discrete frequencies
 *     with the frequency shift of Sec. II.B.
 *
 * Complex data are interleaved (re, im) doubles, fields are [ny][nx] with
 * x contiguous.  Build: gcc -O2 -ffp-contract=off (no fast-math), so every
 * multiply and add rounds as written.
 *
 * Threads: the 2D routines split the independent row transforms, then the
 * independent column transforms, over `threads` POSIX threads.  Each 1D
 * transform is still the plain recursion; threading changes no result.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double re, im;
} cplx;

static const double PI = 3.14159265358979323846264338327950288;

/* ---------------------------------------------------------------------- */
/* 1D: recursive radix-2 decimation in time                                */
/* ---------------------------------------------------------------------- */

/* Transform the n samples in[0], in[stride], ..., in[(n-1)*stride] into
 * out[0..n).  The even-indexed samples are transformed into out[0..n/2),
 * the odd-indexed ones into out[n/2..n), and the two halves are combined
 * with P_k = E_k + w^k O_k, P_{k+n/2} = E_k - w^k O_k (the periodicity of
 * the half-length transforms and w^{k+n/2} = -w^k). */
static void fft_rec(const cplx *in, size_t stride, cplx *out, int n, int sign)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int h = n / 2;
    fft_rec(in, 2 * stride, out, h, sign);
    fft_rec(in + stride, 2 * stride, out + h, h, sign);
    for (int k = 0; k < h; k++) {
        double ang = sign * 2.0 * PI * (double)k / (double)n;
        double wr = cos(ang), wi = sin(ang);
        cplx e = out[k], o = out[k + h];
        double tr = wr * o.re - wi * o.im;
        double ti = wr * o.im + wi * o.re;
        out[k].re = e.re + tr;
        out[k].im = e.im + ti;
        out[k + h].re = e.re - tr;
        out[k + h].im = e.im - ti;
    }
}

static int is_pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }

/* The DFT sum itself for any length n: out[k] = sum_j in[j stride]
 * exp(sign 2 pi i (j k mod n) / n).  The n roots of unity are taken from
 * libm once per line (the same values as per term). */
static void dft_direct(const cplx *in, size_t stride, cplx *out, int n, int sign)
{
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    for (int m = 0; m < n && w; m++) {
        double ang = sign * 2.0 * PI * (double)m / (double)n;
        w[m].re = cos(ang);
        w[m].im = sin(ang);
    }
    for (int k = 0; k < n; k++) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < n; j++) {
            long long m = ((long long)j * k) % n;
            double wr, wi;
            if (w) {
                wr = w[m].re;
                wi = w[m].im;
            } else {
                double ang = sign * 2.0 * PI * (double)m / (double)n;
                wr = cos(ang);
                wi = sin(ang);
            }
            cplx x = in[(size_t)j * stride];
            re += wr * x.re - wi * x.im;
            im += wr * x.im + wi * x.re;
        }
        out[k].re = re;
        out[k].im = im;
    }
    free(w);
}

/* One line: the radix-2 recursion for powers of two, the plain sum else. */
static void transform_line(const cplx *in, size_t stride, cplx *out, int n, int sign)
{
    if (is_pow2(n))
        fft_rec(in, stride, out, n, sign);
    else
        dft_direct(in, stride, out, n, sign);
}

/* Unnormalised 1D transform with exponent sign `sign` (-1 forward, +1 for
 * the unscaled inverse sum), any length n >= 1.  Returns 0, or -1 for a bad
 * argument. */
int oracle_fft1d(const double *in, double *out, int n, int sign)
{
    if (n < 1 || (sign != 1 && sign != -1)) return -1;
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!tmp) return -2;
    transform_line((const cplx *)in, 1, tmp, n, sign);
    memcpy(out, tmp, sizeof(cplx) * (size_t)n);
    free(tmp);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* 2D: rows, then columns                                                  */
/* ---------------------------------------------------------------------- */

typedef struct {
    cplx *data;
    int nx, ny, sign;
    int axis;        /* 0: rows (length nx), 1: columns (length ny) */
    int begin, end;  /* range of lines handled by this worker */
} line_job;

static void *line_worker(void *arg)
{
    line_job *jb = (line_job *)arg;
    int len = jb->axis == 0 ? jb->nx : jb->ny;
    cplx *src = (cplx *)malloc(sizeof(cplx) * (size_t)len);
    cplx *dst = (cplx *)malloc(sizeof(cplx) * (size_t)len);
    if (!src || !dst) {
        free(src);
        free(dst);
        return (void *)1;
    }
    for (int line = jb->begin; line < jb->end; line++) {
        if (jb->axis == 0) {
            cplx *row = jb->data + (size_t)line * jb->nx;
            transform_line(row, 1, dst, len, jb->sign);
            memcpy(row, dst, sizeof(cplx) * (size_t)len);
        } else {
            for (int k = 0; k < len; k++) src[k] = jb->data[(size_t)k * jb->nx + line];
            transform_line(src, 1, dst, len, jb->sign);
            for (int k = 0; k < len; k++) jb->data[(size_t)k * jb->nx + line] = dst[k];
        }
    }
    free(src);
    free(dst);
    return NULL;
}

static int run_lines(cplx *data, int nx, int ny, int sign, int axis, int threads)
{
    int nlines = axis == 0 ? ny : nx;
    if (threads < 1) threads = 1;
    if (threads > nlines) threads = nlines;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    line_job jobs[256];
    int rc = 0;
    for (int t = 0; t < threads; t++) {
        jobs[t].data = data;
        jobs[t].nx = nx;
        jobs[t].ny = ny;
        jobs[t].sign = sign;
        jobs[t].axis = axis;
        jobs[t].begin = (int)((long long)nlines * t / threads);
        jobs[t].end = (int)((long long)nlines * (t + 1) / threads);
    }
    if (threads == 1) return line_worker(&jobs[0]) ? -2 : 0;
    int created[256];
    for (int t = 0; t < threads; t++) {
        created[t] = pthread_create(&tid[t], NULL, line_worker, &jobs[t]) == 0;
        if (!created[t] && line_worker(&jobs[t])) rc = -2;  /* run inline instead */
    }
    for (int t = 0; t < threads; t++) {
        void *ret = NULL;
        if (!created[t]) continue;
        pthread_join(tid[t], &ret);
        if (ret) rc = -2;
    }
    return rc;
}

/* Unnormalised 2D transform, exponent sign `sign`, in -> out (may alias);
 * any nx, ny >= 1. */
int oracle_fft2d(const double *in, double *out, int nx, int ny, int sign, int threads)
{
    if (nx < 1 || ny < 1 || (sign != 1 && sign != -1)) return -1;
    size_t p = (size_t)nx * ny;
    if (out != in) memmove(out, in, sizeof(cplx) * p);
    int rc = run_lines((cplx *)out, nx, ny, sign, 0, threads);
    if (rc) return rc;
    return run_lines((cplx *)out, nx, ny, sign, 1, threads);
}

/* Inverse 2D transform: exp(+2 pi i ...) sum times 1/(nx*ny). */
int oracle_ifft2d(const double *in, double *out, int nx, int ny, int threads)
{
    int rc = oracle_fft2d(in, out, nx, ny, +1, threads);
    if (rc) return rc;
    size_t p = (size_t)nx * ny;
    double s = 1.0 / (double)p;
    for (size_t i = 0; i < 2 * p; i++) out[i] *= s;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Wavenumbers and the three spectral solves                               */
/* ---------------------------------------------------------------------- */

/* Signed index of frequency slot a on an n-point axis: a for a < n/2, else
 * a - n (2a < n also gives 0 on a one-point axis). */
static double signed_index(int a, int n) { return (double)(2 * a < n ? a : a - n); }

/* Angular wavenumber 2 pi a'/L. */
static double wavenumber(int a, int n, double len) { return 2.0 * PI * signed_index(a, n) / len; }

int oracle_solve_poisson(const double *s, double *u, int nx, int ny, double lx, double ly,
                         int threads)
{
    if (lx <= 0 || ly <= 0) return -1;
    size_t p = (size_t)nx * ny;
    cplx *f = (cplx *)malloc(sizeof(cplx) * p);
    if (!f) return -2;
    int rc = oracle_fft2d(s, (double *)f, nx, ny, -1, threads);
    if (rc) {
        free(f);
        return rc;
    }
    for (int b = 0; b < ny; b++) {
        double ky = wavenumber(b, ny, ly);
        for (int a = 0; a < nx; a++) {
            double kx = wavenumber(a, nx, lx);
            double k2 = kx * kx + ky * ky;
            cplx *c = &f[(size_t)b * nx + a];
            if (a == 0 && b == 0) {
                c->re = 0.0;
                c->im = 0.0;
            } else {
                c->re = -c->re / k2;
                c->im = -c->im / k2;
            }
        }
    }
    rc = oracle_ifft2d((double *)f, u, nx, ny, threads);
    free(f);
    return rc;
}

int oracle_solve_diffusion(const double *u0, double *u, int nx, int ny, double lx, double ly,
                           double kappa, double t, int threads)
{
    if (lx <= 0 || ly <= 0 || kappa < 0 || t < 0) return -1;
    size_t p = (size_t)nx * ny;
    cplx *f = (cplx *)malloc(sizeof(cplx) * p);
    if (!f) return -2;
    int rc = oracle_fft2d(u0, (double *)f, nx, ny, -1, threads);
    if (rc) {
        free(f);
        return rc;
    }
    for (int b = 0; b < ny; b++) {
        double ky = wavenumber(b, ny, ly);
        for (int a = 0; a < nx; a++) {
            double kx = wavenumber(a, nx, lx);
            double m = exp(-kappa * (kx * kx + ky * ky) * t);
            cplx *c = &f[(size_t)b * nx + a];
            c->re *= m;
            c->im *= m;
        }
    }
    rc = oracle_ifft2d((double *)f, u, nx, ny, threads);
    free(f);
    return rc;
}

/* Spectra of the wave solution at time t from the spectra F (of u0) and G
 * (of v0, NULL => 0): U = F cos(wt) + G sin(wt)/w, V = -w F sin(wt) + G cos(wt);
 * w = 0: U = F + G t, V = G.  U or V may be NULL. */
int oracle_wave_spectra(const double *F, const double *G, double *U, double *V, int nx, int ny,
                        double lx, double ly, double c, double t)
{
    if (lx <= 0 || ly <= 0 || c < 0) return -1;
    const cplx *Fc = (const cplx *)F, *Gc = (const cplx *)G;
    for (int b = 0; b < ny; b++) {
        double ky = wavenumber(b, ny, ly);
        for (int a = 0; a < nx; a++) {
            double kx = wavenumber(a, nx, lx);
            double w = c * sqrt(kx * kx + ky * ky);
            size_t i = (size_t)b * nx + a;
            cplx f = Fc[i];
            cplx g = Gc ? Gc[i] : (cplx){0.0, 0.0};
            cplx uu, vv;
            if (w == 0.0) {
                uu.re = f.re + g.re * t;
                uu.im = f.im + g.im * t;
                vv = g;
            } else {
                double cs = cos(w * t), sn = sin(w * t);
                uu.re = f.re * cs + g.re * sn / w;
                uu.im = f.im * cs + g.im * sn / w;
                vv.re = -w * f.re * sn + g.re * cs;
                vv.im = -w * f.im * sn + g.im * cs;
            }
            if (U) ((cplx *)U)[i] = uu;
            if (V) ((cplx *)V)[i] = vv;
        }
    }
    return 0;
}

int oracle_solve_wave(const double *u0, const double *v0, double *u, double *v, int nx, int ny,
                      double lx, double ly, double c, double t, int threads)
{
    if (lx <= 0 || ly <= 0 || c < 0) return -1;
    size_t p = (size_t)nx * ny;
    cplx *F = (cplx *)malloc(sizeof(cplx) * p);
    cplx *G = v0 ? (cplx *)malloc(sizeof(cplx) * p) : NULL;
    cplx *U = (cplx *)malloc(sizeof(cplx) * p);
    cplx *V = v ? (cplx *)malloc(sizeof(cplx) * p) : NULL;
    int rc = -2;
    if (!F || !U || (v0 && !G) || (v && !V)) goto done;
    rc = oracle_fft2d(u0, (double *)F, nx, ny, -1, threads);
    if (!rc && v0) rc = oracle_fft2d(v0, (double *)G, nx, ny, -1, threads);
    if (!rc)
        rc = oracle_wave_spectra((double *)F, (double *)G, (double *)U, (double *)V, nx, ny, lx, ly,
                                 c, t);
    if (!rc) rc = oracle_ifft2d((double *)U, u, nx, ny, threads);
    if (!rc && v) rc = oracle_ifft2d((double *)V, v, nx, ny, threads);
done:
    free(F);
    free(G);
    free(U);
    free(V);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Time-independent sources                                                */
/* ---------------------------------------------------------------------- */

/* Diffusion with a source constant in time (Sec. III.B): each coefficient
 * obeys du^/dt = -kappa|k|^2 u^ + s^ (Eq. (DiffusionIVPFS) with diffusivity
 * kappa), u^(0) = f^, so with q = kappa|k|^2
 *   u^(t) = f^ exp(-q t) + s^ (1 - exp(-q t)) / q     (q > 0)
 *   u^(t) = f^ + s^ t                                  (q = 0). */
int oracle_solve_diffusion_source(const double *f, const double *s, double *u, int nx, int ny,
                                  double lx, double ly, double kappa, double t, int threads)
{
    if (lx <= 0 || ly <= 0 || kappa < 0 || t < 0) return -1;
    size_t p = (size_t)nx * ny;
    cplx *F = (cplx *)malloc(sizeof(cplx) * p);
    cplx *S = (cplx *)malloc(sizeof(cplx) * p);
    int rc = -2;
    if (!F || !S) goto done;
    rc = oracle_fft2d(f, (double *)F, nx, ny, -1, threads);
    if (!rc) rc = oracle_fft2d(s, (double *)S, nx, ny, -1, threads);
    if (rc) goto done;
    for (int b = 0; b < ny; b++) {
        double ky = wavenumber(b, ny, ly);
        for (int a = 0; a < nx; a++) {
            double kx = wavenumber(a, nx, lx);
            double q = kappa * (kx * kx + ky * ky);
            size_t i = (size_t)b * nx + a;
            double e, m;
            if (q == 0.0) {
                e = 1.0;
                m = t;
            } else {
                e = exp(-q * t);
                m = (1.0 - e) / q;
            }
            F[i].re = F[i].re * e + S[i].re * m;
            F[i].im = F[i].im * e + S[i].im * m;
        }
    }
    rc = oracle_ifft2d((double *)F, u, nx, ny, threads);
done:
    free(F);
    free(S);
    return rc;
}

/* Wave with a source constant in time (Sec. III.C): each coefficient is a
 * forced oscillator u^'' + w^2 u^ = s^ (Eq. (WaveEquationFourierSpace)),
 * u^(0) = f^, u^'(0) = g^, w = c|k|:
 *   w = 0:  u^ = s^ t^2/2 + g^ t + f^                    (Eq. (OmegaZero))
 *           v^ = s^ t + g^
 *   w > 0:  u^ = (f^ - s^/w^2) cos(w t) + g^ sin(w t)/w + s^/w^2
 *           v^ = -w (f^ - s^/w^2) sin(w t) + g^ cos(w t)
 * The constant particular solution s^/w^2 is written out here; Eq.
 * (OmegaNonZero) as printed leaves it out, and without it u^ would not
 * satisfy the oscillator equation.  g, v may be NULL (g = 0; no velocity). */
int oracle_solve_wave_source(const double *f, const double *g, const double *s, double *u, double *v,
                             int nx, int ny, double lx, double ly, double c, double t, int threads)
{
    if (lx <= 0 || ly <= 0 || c < 0) return -1;
    size_t p = (size_t)nx * ny;
    cplx *F = (cplx *)malloc(sizeof(cplx) * p);
    cplx *G = g ? (cplx *)malloc(sizeof(cplx) * p) : NULL;
    cplx *S = (cplx *)malloc(sizeof(cplx) * p);
    cplx *V = v ? (cplx *)malloc(sizeof(cplx) * p) : NULL;
    int rc = -2;
    if (!F || !S || (g && !G) || (v && !V)) goto done;
    rc = oracle_fft2d(f, (double *)F, nx, ny, -1, threads);
    if (!rc && g) rc = oracle_fft2d(g, (double *)G, nx, ny, -1, threads);
    if (!rc) rc = oracle_fft2d(s, (double *)S, nx, ny, -1, threads);
    if (rc) goto done;
    for (int b = 0; b < ny; b++) {
        double ky = wavenumber(b, ny, ly);
        for (int a = 0; a < nx; a++) {
            double kx = wavenumber(a, nx, lx);
            double w = c * sqrt(kx * kx + ky * ky);
            size_t i = (size_t)b * nx + a;
            cplx ff = F[i], ss = S[i];
            cplx gg = G ? G[i] : (cplx){0.0, 0.0};
            cplx uu, vv;
            if (w == 0.0) {
                uu.re = ss.re * t * t / 2.0 + gg.re * t + ff.re;
                uu.im = ss.im * t * t / 2.0 + gg.im * t + ff.im;
                vv.re = ss.re * t + gg.re;
                vv.im = ss.im * t + gg.im;
            } else {
                double cs = cos(w * t), sn = sin(w * t), w2 = w * w;
                cplx h = {ff.re - ss.re / w2, ff.im - ss.im / w2};
                uu.re = h.re * cs + gg.re * sn / w + ss.re / w2;
                uu.im = h.im * cs + gg.im * sn / w + ss.im / w2;
                vv.re = -w * h.re * sn + gg.re * cs;
                vv.im = -w * h.im * sn + gg.im * cs;
            }
            F[i] = uu;
            if (V) V[i] = vv;
        }
    }
    rc = oracle_ifft2d((double *)F, u, nx, ny, threads);
    if (!rc && v) rc = oracle_ifft2d((double *)V, v, nx, ny, threads);
done:
    free(F);
    free(G);
    free(S);
    free(V);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* 3D (the n-dimensional extension of Sec. II.D): x lines, y lines, z lines */
/* ---------------------------------------------------------------------- */

/* Unnormalised 3D transform of a [nz][ny][nx] field, exponent sign `sign`:
 * the 2D transform of every z plane, then every z line, the latter seen as
 * the columns of an [nz][nx*ny] array. */
int oracle_fft3d(const double *in, double *out, int nx, int ny, int nz, int sign, int threads)
{
    if (!is_pow2(nx) || !is_pow2(ny) || !is_pow2(nz) || (sign != 1 && sign != -1)) return -1;
    size_t plane = (size_t)nx * ny, p = plane * nz;
    if (out != in) memmove(out, in, sizeof(cplx) * p);
    for (int z = 0; z < nz; z++) {
        cplx *pl = (cplx *)out + plane * z;
        int rc = run_lines(pl, nx, ny, sign, 0, threads);
        if (!rc) rc = run_lines(pl, nx, ny, sign, 1, threads);
        if (rc) return rc;
    }
    return run_lines((cplx *)out, nx * ny, nz, sign, 1, threads);
}

int oracle_ifft3d(const double *in, double *out, int nx, int ny, int nz, int threads)
{
    int rc = oracle_fft3d(in, out, nx, ny, nz, +1, threads);
    if (rc) return rc;
    size_t p = (size_t)nx * ny * nz;
    double s = 1.0 / (double)p;
    for (size_t i = 0; i < 2 * p; i++) out[i] *= s;
    return 0;
}

/* The three solves on a periodic lx-by-ly-by-lz box, |k|^2 = kx^2 + ky^2 +
 * kz^2: op 0 Poisson (-1/|k|^2, k = 0 -> 0), op 1 diffusion
 * (exp(-kappa |k|^2 t)), op 2 wave with zero initial velocity (cos(c|k|t)). */
int oracle_solve3d(const double *in, double *out, int nx, int ny, int nz, double lx, double ly, double lz,
                   int op, double coef, double t, int threads)
{
    if (lx <= 0 || ly <= 0 || lz <= 0 || op < 0 || op > 2) return -1;
    size_t plane = (size_t)nx * ny, p = plane * nz;
    cplx *f = (cplx *)malloc(sizeof(cplx) * p);
    if (!f) return -2;
    int rc = oracle_fft3d(in, (double *)f, nx, ny, nz, -1, threads);
    if (rc) {
        free(f);
        return rc;
    }
    for (int z = 0; z < nz; z++) {
        double kz = wavenumber(z, nz, lz);
        for (int b = 0; b < ny; b++) {
            double ky = wavenumber(b, ny, ly);
            for (int a = 0; a < nx; a++) {
                double kx = wavenumber(a, nx, lx);
                double k2 = kx * kx + ky * ky + kz * kz;
                double m;
                if (op == 0) m = (a == 0 && b == 0 && z == 0) ? 0.0 : -1.0 / k2;
                else if (op == 1) m = exp(-coef * k2 * t);
                else m = cos(coef * sqrt(k2) * t);
                cplx *c = &f[plane * z + (size_t)b * nx + a];
                c->re *= m;
                c->im *= m;
            }
        }
    }
    rc = oracle_ifft3d((double *)f, out, nx, ny, nz, threads);
    free(f);
    return rc;
}
