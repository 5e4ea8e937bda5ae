/*
 * fftpde.h -- C ABI of libfftpde.so: 2D FFTs and FFT spectral solves of the
 * periodic Poisson, diffusion and wave equations on one AMD Instinct MI355X
 * (gfx950) GPU.  Method: arXiv 2412.12308, "Numerical Solution of Partial
 * Differential Equations using the Discrete Fourier Transform".
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  Fields.  Complex, interleaved (re, im).  FFTPDE_C64 = FP32 complex
 *    (8 bytes per point), FFTPDE_C128 = FP64 complex (16 bytes per point).
 *    A field is nx*ny points stored row-major as [ny][nx] with x contiguous:
 *    point (x_j, y_k) is element k*nx + j.  A batch of `batch` fields is
 *    stored back to back (field b starts at element b*nx*ny).  Sampling
 *    follows Sec. II.B/II.D: x_j = x0 + j*lx/nx, j = 0..nx-1 (periodic,
 *    endpoint excluded); the origin x0 never enters a solve.
 *  Sizes.  nx and ny are powers of two in [2, 4096] (the FFT's 2^m
 *    restriction, Sec. II.C); batch >= 1.  fft2d_forward, fft2d_inverse,
 *    fft2d_r2c, fft2d_c2r, solve_poisson, solve_diffusion and solve_wave
 *    also take sides that are not powers of two: any side in [2, 4096]
 *    whose prime factors are 2, 3, 5 and 7 (the mixed-radix path: Stockham
 *    stages of radix 2, 3, 4, 5, 7 and 8, an extension of Sec. II.D; EINVAL
 *    for other sides), with the same dtypes as on powers of two (real
 *    fields in pairs; the workspace holds the pair spectra).  The first
 *    call for a new side allocates and uploads that length's twiddle table
 *    (kept until the context is destroyed).  Every other entry point takes
 *    powers of two only.
 *  Pointers.  Every field pointer is a DEVICE pointer on the context's GPU,
 *    aligned to the element size.  The caller owns every field buffer.
 *    in == out (in place) is allowed wherever an input and an output have the
 *    same size; other partial overlaps are not.
 *  Streams.  `stream` is a hipStream_t (NULL = the legacy default stream).
 *    Calls only enqueue work: outputs are valid once the stream has reached
 *    the call.  Calls on one context from several host threads must be
 *    serialised by the caller.
 *  Transform sign.  Forward = exp(-2 pi i (a j/nx + b k/ny)), unnormalised;
 *    inverse = exp(+2 pi i ...) times 1/(nx ny).  This is the sign of the
 *    row-column derivation of Sec. II.D; the paper's Eq. (DFT) writes the
 *    opposite sign, which only reverses the frequency index and leaves every
 *    solve below unchanged (their symbols are even in k).
 *  Wavenumbers.  k_x = 2 pi a'/lx with a' = a for 2a < nx, else a - nx
 *    (the shifted frequencies of Sec. II.B and II.D; a = nx/2 gives -nx/2
 *    on even sides, odd sides have no such slot); likewise k_y;
 *    |k|^2 = k_x^2 + k_y^2.
 *  Status.  Every function returns an int status (FFTPDE_OK = 0, negative =
 *    error); no C++ exception crosses this boundary.  Arguments are checked
 *    before any device work; a rejected call enqueues nothing.
 *    FFTPDE_EDEVICE may report an earlier asynchronous launch failure.
 */
#ifndef FFTPDE_H
#define FFTPDE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FFTPDE_OK 0
#define FFTPDE_PENDING 1      /* serving: request not finished yet */
#define FFTPDE_EINVAL (-1)    /* bad size, pointer, dtype or coefficient */
#define FFTPDE_ENOMEM (-2)    /* host or device allocation failed */
#define FFTPDE_EDEVICE (-3)   /* a HIP call or kernel launch failed */
#define FFTPDE_EBUDGET (-4)   /* serving: request larger than the whole budget */
#define FFTPDE_ENOTFOUND (-5) /* unknown request id or plan */
#define FFTPDE_ECANCELED (-6) /* serving: request cancelled */
#define FFTPDE_ETIMEOUT (-7)  /* serving: deadline passed before completion */

/* ---- dtypes and operators ---------------------------------------------- */
#define FFTPDE_C64 0  /* FP32 complex; FP64 twiddles rounded once, FP64 phases */
#define FFTPDE_C128 1 /* FP64 complex throughout */
/* Real fields (the 2D solves, the sourced solves and the half-spectrum
 * transforms): FP32 / FP64 points, batch*nx*ny values per
 * buffer, same row-major layout.  The solves' symbols are real and even in k,
 * so a solve maps real fields to real fields and S(u1 + i u2) = S(u1) +
 * i S(u2): fields 2p and 2p+1 of the batch are solved together as the real
 * and imaginary parts of one complex field (an odd last field is paired
 * with zero), in the precision of FFTPDE_C64 / FFTPDE_C128.  Each real field
 * moves half the bytes of a complex one.  The rounding error of a field is
 * bounded relative to the norm of its pair (sqrt(|u1|^2 + |u2|^2)), not its
 * own norm alone.  fft2d_forward / fft2d_inverse, 3D, RK4, evolution,
 * batches and the server take complex fields only. */
#define FFTPDE_R32 2
#define FFTPDE_R64 3

#define FFTPDE_POISSON 0   /* lap(u) = s                  (Sec. III.A) */
#define FFTPDE_DIFFUSION 1 /* u_t = kappa lap(u)          (Sec. III.B) */
#define FFTPDE_WAVE 2      /* u_tt = c^2 lap(u)           (Sec. III.C) */

typedef void *fftpde_stream; /* a hipStream_t */
typedef struct fftpde_ctx fftpde_ctx;
typedef struct fftpde_evolve fftpde_evolve;
typedef struct fftpde_batch fftpde_batch;
typedef struct fftpde_server fftpde_server;

/* ---- lifecycle ----------------------------------------------------------
 * fftpde_create: make `device` current, build the twiddle tables
 *   w^e = exp(-2 pi i e/4096), e = 0..4095, in FP64 on the host and round them
 *   once to FP32 for the C64 table (the w_N^k of Sec. II.B/II.C; a length-N
 *   transform reads every (4096/N)-th entry), and upload both.  *ctx receives
 *   an opaque handle owned by the caller until fftpde_destroy.
 * fftpde_destroy: frees everything the context owns (tables, plan cache,
 *   workspace); NULL is accepted.  The caller must first finish or destroy
 *   evolutions, batches and servers made from it.
 * fftpde_strerror: static text for a status code, never NULL.
 * fftpde_version: library version string. */
int fftpde_create(fftpde_ctx **ctx, int device);
int fftpde_destroy(fftpde_ctx *ctx);
const char *fftpde_strerror(int status);
const char *fftpde_version(void);
/* fftpde_last_error: text of the last HIP failure seen by this host thread
 * (the detail behind an FFTPDE_EDEVICE), "" if none; valid until the next
 * call on the same thread. */
const char *fftpde_last_error(void);

/* ---- kernel timing ------------------------------------------------------
 * fftpde_profile: enable (1) or disable (0) timing of every kernel this
 *   context launches from now on; either call drops earlier records.  Each
 *   launch is bracketed by two HIP events recorded on the launch's stream.
 * fftpde_profile_read: wait for the recorded launches and write a JSON array
 *   [{"kernel": name, "launches": n, "total_ms": t, "bytes": b}, ...] into
 *   buf (cap bytes, NUL-terminated), where b is the algorithmic HBM traffic
 *   (each field read once and written once per launch).  *needed (if not
 *   NULL) receives the size required; a too-small buf gives FFTPDE_ENOMEM. */
int fftpde_profile(fftpde_ctx *ctx, int enable);
int fftpde_profile_read(fftpde_ctx *ctx, char *buf, size_t cap, size_t *needed);

/* ---- kernel plans -------------------------------------------------------
 * Every pass is one of several compiled kernel variants (radix schedule,
 * tile width, threads, LDS exchange, prefetch); each (dtype, pass, length,
 * fields) slot has a default.
 * fftpde_plan_variants: JSON array describing every compiled variant
 *   ({"name", "dtype", "pass", "logn", "fields", ..., "active"}), written
 *   like fftpde_profile_read.
 * fftpde_plan_select: make the named variant the one used for its slot on
 *   this context (FFTPDE_ENOTFOUND if no such name); NULL or "" restores every
 *   slot's default.  Every variant computes the same transform; they differ
 *   in speed and in rounding order only. */
int fftpde_plan_variants(fftpde_ctx *ctx, char *buf, size_t cap, size_t *needed);
int fftpde_plan_select(fftpde_ctx *ctx, const char *name);
/* fftpde_plan_small: enable (default) or disable the single-pass small-grid
 *   path: for the grids it is compiled for (both sides in [32, 512] with at most
 *   16384 points in C64, [32, 256] and 8192 points in C128) a transform or a
 *   single-field solve is one launch, one workgroup per field holding the
 *   field in LDS (one HBM read and one write). */
int fftpde_plan_small(fftpde_ctx *ctx, int enable);
/* fftpde_plan_tiled: the layout of the spectrum between the passes of the
 *   3-pass solves without an initial velocity.  block_bytes > 0 (default
 *   1024): the forward row pass writes it into a scratch field of the context
 *   (one per stream, grown on demand, freed by fftpde_destroy) in column
 *   blocks of block_bytes per row (at least one column tile wide) x ny rows,
 *   the column pass reads and writes within contiguous blocks, and the
 *   inverse row pass writes the row-major result; 0: row-major in the output
 *   field.  Results are bit-identical for every block size; only the memory
 *   access pattern changes.  EINVAL unless 0 or a power of two <= 65536. */
int fftpde_plan_tiled(fftpde_ctx *ctx, int block_bytes);
/* fftpde_plan_chunk: a batch of 3-pass solves without an initial velocity
 *   runs in chunks of about `bytes` of field data (at least one field), all
 *   three passes of a chunk before the next, so that the spectrum one pass
 *   writes is still in the GPU's 256 MiB Infinity Cache when the next pass
 *   reads it.  Default 256 MiB; 0 = the whole batch at once.  Real fields
 *   (solved in pairs) count their pair spectra twice, so a chunk holds half
 *   as many pairs (not so the inverse half transform fft2d_c2r).  Results
 *   are bit-identical for every chunk size.  EINVAL for negative sizes. */
int fftpde_plan_chunk(fftpde_ctx *ctx, long long bytes);

/* fftpde_autotune: for an (nx, ny, batch, dtype, op) solve (op one of
 *   FFTPDE_POISSON / DIFFUSION / WAVE, zero initial velocity), time every
 *   compiled variant of the row pass for nx and of the column pass for ny on
 *   library-owned scratch fields filled with a fixed pseudo-random pattern,
 *   `reps` timed solves each (HIP events on `stream`).  A variant is admitted
 *   only if its result matches the plan in use at the call to relative L2
 *   <= 1e-12 (C128) or 2 * 2e-6 * log2(max(nx, ny)) (C64); the fastest admitted
 *   variant becomes this context's plan for its slot.  Then, for shapes that
 *   take the 3-pass path, the layout of the spectrum between the passes
 *   (fftpde_plan_tiled block sizes 0, 256, 1024, 4096) is timed the same way
 *   and the fastest admitted one is kept for this shape and dtype, and so is
 *   the chunk size of the batch (fftpde_plan_chunk: 0, 64, 128, 256, 512
 *   MiB).  A JSON report ({"candidates": [{"name", "pass", "us", "err",
 *   "ok"}], "tiled_bytes", "chunk_bytes" (-1 if not tuned), "row", "col"})
 *   is written like
 *   fftpde_profile_read (report may be NULL).  Synchronises the stream;
 *   allocates and frees 3 * batch * nx * ny elements of scratch.
 * fftpde_plan_save / fftpde_plan_load: write / apply the plan of this
 *   context as a text file: one variant name per line, and one line
 *   "tiled <dtype> <log2 nx> <log2 ny> <block bytes>" / "chunk <dtype>
 *   <log2 nx> <log2 ny> <bytes>" per tuned layout / chunk size ('#'
 *   comments).  Loading a name that is not compiled in gives
 *   FFTPDE_ENOTFOUND, a malformed layout or chunk line FFTPDE_EINVAL (the
 *   other lines still apply).  fftpde_plan_select(ctx, NULL) drops tuned
 *   layouts and chunk sizes; fftpde_plan_tiled / fftpde_plan_chunk drop the
 *   tuned ones of their kind. */
int fftpde_autotune(fftpde_ctx *ctx, int nx, int ny, int batch, int dtype, int op, int reps,
                    fftpde_stream stream, char *report, size_t cap, size_t *needed);
int fftpde_plan_save(fftpde_ctx *ctx, const char *path);
int fftpde_plan_load(fftpde_ctx *ctx, const char *path);

/* ---- 2D transforms (Sec. II.D, Eq. (2D_DFT); iDFT of Sec. II.B) ----------
 * fft2d_forward: out = unnormalised forward 2D transform of in, for each of
 *   `batch` fields.  Done as all x-direction (row) transforms for fixed y,
 *   then all y-direction (column) transforms for fixed x frequency.
 * fft2d_inverse: out = exp(+) transform times 1/(nx ny).
 *   in/out: device fields of the given dtype, batch*nx*ny points each. */
int fft2d_forward(fftpde_ctx *ctx, const void *in, void *out, int nx, int ny, int batch,
                  int dtype, fftpde_stream stream);
int fft2d_inverse(fftpde_ctx *ctx, const void *in, void *out, int nx, int ny, int batch,
                  int dtype, fftpde_stream stream);

/* ---- 2D transforms of real fields (half spectra) ----------------------------
 * The transform of real data has X[-b][-a] = conj(X[b][a]) (Sec. II.B), so
 * columns a = 0 .. nx/2 of the spectrum determine it: the half spectrum, a
 * [ny][nx/2 + 1] complex field (nx/2 rounded down: columns 0 .. (nx-1)/2
 * on odd sides).
 * fft2d_r2c: out = the half spectrum (unnormalised forward transform) of
 *   each real field of `in`.  dtype FFTPDE_R32 (in: float, out: FP32
 *   complex) or FFTPDE_R64 (double / FP64 complex); sides in [2, 4096],
 *   powers of two or 7-smooth.
 * fft2d_c2r: out = the real field whose half spectrum is the Hermitian part
 *   of `in`, times 1/(nx ny): columns 0 < a < nx/2 as given, the rest of the
 *   spectrum from the symmetry, and the self-conjugate columns (a = 0, and
 *   a = nx/2 on even nx) replaced by (X[b][a] + conj(X[-b][a]))/2 (no change
 *   for half spectra of real fields).  Same dtypes and sides.
 * Both: in and out must not overlap (EINVAL).  Powers of two with nx, ny
 *   >= 16 (and nx ny >= 2^15 FP32 / 2^14 FP64), the real side aligned to a
 *   complex element: each real field is read as a complex field of nx/2
 *   columns, its column transforms go to the per-stream scratch, and a row
 *   pass over row pairs (b, -b) transforms the rows and splits them into
 *   whole half-spectrum rows by the even/odd combination of Sec. II.C
 *   (c2r: the same steps backwards).  Other shapes: two real fields go
 *   through one complex transform, their spectrum in the per-stream
 *   scratch; one more pass splits it into the two half spectra (or joins
 *   them). */
int fft2d_r2c(fftpde_ctx *ctx, const void *in, void *out, int nx, int ny, int batch, int dtype,
              fftpde_stream stream);
int fft2d_c2r(fftpde_ctx *ctx, const void *in, void *out, int nx, int ny, int batch, int dtype,
              fftpde_stream stream);

/* ---- spectral solves ----------------------------------------------------
 * Each is forward 2D FFT -> pointwise multiply by the equation's Fourier
 * symbol -> inverse 2D FFT.  The multiply and the 1/(nx ny) of the inverse
 * run inside the column pass, between its forward and inverse transforms.
 *
 * solve_poisson: lap(u) = s on a periodic lx-by-ly box (Eq. (Poisson)).
 *   The mean of s is removed (g = s - mean(s), Eq. (Poisson2)) by dropping the
 *   k = 0 coefficient, and u is the zero-mean solution
 *   u = F^-1{ -F{g} / |k|^2 } (Eq. (SolutionPoisson)) with u^(0) = 0.
 *   s: input fields, u: output fields (may equal s).
 * solve_diffusion: u(t) for u_t = kappa lap(u), u(0) = u0, source-free
 *   (Eq. (EcuacionDeCalor) with diffusivity kappa):
 *   u^(t) = u0^ exp(-kappa |k|^2 t) (Eq. (solCalorFourier)).  kappa >= 0,
 *   t >= 0 (the backward heat equation is rejected), both finite.  The
 *   exponent kappa |k|^2 t is formed in FP64 for both dtypes.
 * solve_wave: u(t) (and u_t(t)) for u_tt = c^2 lap(u), u(0) = u0,
 *   u_t(0) = v0, source-free (Eq. (wave_equation), (OndaCI)):
 *   u^ = u0^ cos(w t) + v0^ sin(w t)/w with w = c|k|, and u0^ + v0^ t at
 *   w = 0 (Eq. (OmegaNonZero), (OmegaZero) with s = 0); the velocity is
 *   v^ = -w u0^ sin(w t) + v0^ cos(w t).  v0 = NULL means v0 = 0; v = NULL
 *   means the velocity is not written.  c >= 0, t any finite value (negative
 *   t runs the wave backwards).  The phase w t is formed and reduced in FP64
 *   for both dtypes. */
int solve_poisson(fftpde_ctx *ctx, const void *s, void *u, int nx, int ny, int batch, double lx,
                  double ly, int dtype, fftpde_stream stream);
int solve_diffusion(fftpde_ctx *ctx, const void *u0, void *u, int nx, int ny, int batch,
                    double lx, double ly, double kappa, double t, int dtype,
                    fftpde_stream stream);
int solve_wave(fftpde_ctx *ctx, const void *u0, const void *v0, void *u, void *v, int nx, int ny,
               int batch, double lx, double ly, double c, double t, int dtype,
               fftpde_stream stream);

/* ---- a solve that allocates nothing --------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * solve_wave_noalloc: solve_wave (same arguments, meaning and results, bit
 *   for bit) on complex fields (FFTPDE_C64 / FFTPDE_C128) whose sides are
 *   powers of two, with the spectrum between its passes kept in a fixed
 *   device array of FFTPDE_NOALLOC_SCRATCH_BYTES that the library holds on
 *   every GPU it runs on until the process ends, instead of the context's
 *   workspace; it calls no hipMalloc or hipFree.  Batches run in chunks of
 *   as many fields as the array holds.  A side or dtype that solve_wave takes
 *   but this does not, or a field whose spectrum (two with a velocity input
 *   or output) exceeds the array, is rejected with FFTPDE_EINVAL before any
 *   work is enqueued (fftpde_last_error says which); FFTPDE_EDEVICE if the
 *   array's address could not be found at fftpde_create.  Every call on one
 *   GPU uses the same array: calls that overlap in time on one GPU (other
 *   streams, other contexts or threads) race and must be serialised by the
 *   caller. */
#define FFTPDE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int solve_wave_noalloc(fftpde_ctx *ctx, const void *u0, const void *v0, void *u, void *v, int nx, int ny,
                       int batch, double lx, double ly, double c, double t, int dtype, fftpde_stream stream);

/* ---- sources constant in time ------------------------------------------
 * solve_diffusion_source: u(t) for u_t = kappa lap(u) + s, u(0) = f, with s
 *   independent of t (Sec. III.B, Eq. (DiffusionIVPFS) with diffusivity
 *   kappa): per coefficient, with q = kappa |k|^2,
 *     u^ = f^ exp(-q t) + s^ (1 - exp(-q t))/q,   and f^ + s^ t at q = 0.
 *   kappa >= 0, t >= 0 finite.
 * solve_wave_source: u(t) (and u_t(t)) for u_tt = c^2 lap(u) + s, u(0) = f,
 *   u_t(0) = g, s independent of t (Sec. III.C): per coefficient the forced
 *   oscillator, w = c|k|,
 *     u^ = (f^ - s^/w^2) cos(w t) + g^ sin(w t)/w + s^/w^2,
 *     v^ = -w (f^ - s^/w^2) sin(w t) + g^ cos(w t),
 *   and s^ t^2/2 + g^ t + f^ (Eq. (OmegaZero)), v^ = s^ t + g^ at w = 0.  The
 *   constant particular solution s^/w^2 completes Eq. (OmegaNonZero), which
 *   prints the solution without it.  g = NULL means g = 0; v = NULL means
 *   the velocity is not written; v must differ from u.  c >= 0, t finite.
 * Both: complex or real dtypes (real fields in pairs, see FFTPDE_R32); the
 *   oscillator's cos, sin and (1 - cos(w t))/w^2 = 2 sin^2(w t/2)/w^2, and
 *   the decay's exp(-q t) and its expm1 form, take FP64 arguments for every
 *   dtype.  Three row passes in (two without g), one column pass, one or two
 *   out; the spectra between them live in the context's per-stream scratch
 *   (two or three fields per 256 MiB chunk of fields).  An output may be the
 *   same buffer as an input. */
int solve_diffusion_source(fftpde_ctx *ctx, const void *f, const void *s, void *u, int nx, int ny,
                           int batch, double lx, double ly, double kappa, double t, int dtype,
                           fftpde_stream stream);
int solve_wave_source(fftpde_ctx *ctx, const void *f, const void *g, const void *s, void *u, void *v,
                      int nx, int ny, int batch, double lx, double ly, double c, double t, int dtype,
                      fftpde_stream stream);

/* ---- 3D ------------------------------------------------------------------
 * Fields [nz][ny][nx] (x contiguous, then y, then z), nx, ny, nz powers of
 * two in [2, 4096] with nx*ny <= 2^24; batch fields back to back; complex
 * dtypes.  The transform is the n-dimensional extension of the row-column
 * scheme of Sec. II.D: x rows, then the y columns of every z plane, then the
 * z columns.  fft3d_inverse scales by 1/(nx ny nz).  The solves are those of
 * the 2D entry points with |k|^2 = kx^2 + ky^2 + kz^2 (the wave without an
 * initial velocity), five passes: x, y, z with the symbol fused between its
 * forward and inverse transforms, y, x.  In place allowed. */
int fft3d_forward(fftpde_ctx *ctx, const void *in, void *out, int nx, int ny, int nz, int batch,
                  int dtype, fftpde_stream stream);
int fft3d_inverse(fftpde_ctx *ctx, const void *in, void *out, int nx, int ny, int nz, int batch,
                  int dtype, fftpde_stream stream);
int solve_poisson_3d(fftpde_ctx *ctx, const void *s, void *u, int nx, int ny, int nz, int batch,
                     double lx, double ly, double lz, int dtype, fftpde_stream stream);
int solve_diffusion_3d(fftpde_ctx *ctx, const void *u0, void *u, int nx, int ny, int nz, int batch,
                       double lx, double ly, double lz, double kappa, double t, int dtype,
                       fftpde_stream stream);
int solve_wave_3d(fftpde_ctx *ctx, const void *u0, void *u, int nx, int ny, int nz, int batch,
                  double lx, double ly, double lz, double c, double t, int dtype,
                  fftpde_stream stream);

/* ---- a source that depends on time: RK4 in Fourier space ----------------
 * fftpde_wave_rk4: (u, u_t) at t0 + steps*dt for u_tt = c^2 lap(u) + s(t),
 *   u(t0) = f, u_t(t0) = g (NULL => 0), with the orbiting Gaussian source of
 *   Sec. III.C,
 *     s(t, x, y) = A exp(-d^2/sigma^2) cos(gamma t),
 *   d the periodic (minimum-image) distance from (x, y) to the centre
 *   (cx + r cos(Omega t), cy + r sin(Omega t)).  The grid is
 *   x_j = x0 + j lx/nx, y_k = y0 + k ly/ny (the origin matters here: the
 *   source sits at absolute positions).  Every Fourier coefficient of the
 *   first-order system u^' = v^, v^' = -w^2 u^ + s^(t) (w = c|k|) advances
 *   by the classical fourth-order Runge-Kutta method with step dt; the
 *   source is sampled on the grid and transformed at t, t + dt/2 and t + dt
 *   of each step (the transform at t + dt serves the next step).  The
 *   spectra live in the context's per-stream scratch ((2 batch + 3) fields)
 *   between the calls' kernels; the batch shares the source.  Complex
 *   dtypes.  sigma > 0; A, r, Omega, gamma, cx, cy, x0, y0, t0, dt finite;
 *   c >= 0; steps >= 0; v may be NULL (not written) and must differ from u.
 *   The method is stable for c |k|_max |dt| below about 2.8. */
typedef struct {
  double amplitude; /* A */
  double sigma;     /* width sigma_s */
  double radius;    /* orbit radius r_s */
  double omega;     /* orbit angular frequency Omega */
  double gamma;     /* angular frequency gamma of the amplitude */
  double cx, cy;    /* orbit centre */
} fftpde_orbit_source;
int fftpde_wave_rk4(fftpde_ctx *ctx, const fftpde_orbit_source *src, const void *f, const void *g,
                    void *u, void *v, int nx, int ny, int batch, double x0, double y0, double lx,
                    double ly, double c, double t0, double dt, int steps, int dtype,
                    fftpde_stream stream);

/* ---- time evolution with resident spectra -------------------------------
 * The diffusion and wave solutions are closed forms in time
 * (Eq. (solCalorFourier); Eq. (OmegaNonZero), (OmegaZero) with s = 0), so a
 * time step is an evaluation at the absolute time t_n = n * dt (one FP64
 * product; nothing accumulates over steps), as the paper's snapshots are.
 *
 * fftpde_evolve_create: kind = FFTPDE_DIFFUSION (coef = kappa >= 0; v0 must be
 *   NULL) or FFTPDE_WAVE (coef = c >= 0; v0 = initial velocity or NULL for 0).
 *   Computes and keeps on the device the forward spectra of u0 (and v0) for
 *   `batch` fields: the library owns batch*nx*ny elements per spectrum until
 *   fftpde_evolve_destroy.  u0/v0 are only read (stream-ordered) and may be
 *   reused once the stream has passed this call.
 * fftpde_evolve_step: state at t = n * dt.  u (may be NULL) receives u(t);
 *   v (wave only, requires u, may be NULL) receives u_t(t).  diag (a DEVICE
 *   array of 3*batch doubles, may be NULL) receives per field the mean of u(t)
 *   (real, imaginary part: the k = 0 coefficient over nx*ny, conserved as in
 *   the paper's Sec. III.B/III.C plots) and an energy computed from the
 *   spectra in FP64 (Parseval): diffusion integral |u|^2 dx dy; wave
 *   1/2 integral (|u_t|^2 + c^2 |grad u|^2) dx dy.  Diffusion requires t >= 0.
 *   A step with u = NULL only reads the spectra (diagnostics).
 * fftpde_evolve_destroy: waits for the device, frees the spectra; NULL ok. */
int fftpde_evolve_create(fftpde_ctx *ctx, int kind, const void *u0, const void *v0, int nx, int ny,
                         int batch, double lx, double ly, double coef, int dtype,
                         fftpde_stream stream, fftpde_evolve **ev);
int fftpde_evolve_step(fftpde_evolve *ev, long long n, double dt, void *u, void *v, double *diag,
                       fftpde_stream stream);
int fftpde_evolve_destroy(fftpde_evolve *ev);

/* ---- batches of uneven solves ---------------------------------------------
 * Many independent solves of different power-of-two shapes, operators, boxes
 * and times (the per-field work of Sec. III, for many small and medium
 * fields at once) as ONE persistent kernel: every job is a row pass, a fused
 * column pass (forward y FFT, symbol, inverse y FFT) and an inverse row pass,
 * cut into tiles of 8192 (FP32) / 4096 (FP64) points; workgroups take tiles
 * from one queue and a job's column tiles start as soon as its own row tiles
 * are done.  A job whose field fits one tile (nx*ny <= 8192 FP32 / 4096
 * FP64) is instead solved in one pass, all five steps in LDS, up to
 * tile/(nx*ny) jobs of one shape and operator per queue item (one HBM read
 * and one write per field).  Each job is computed exactly as the
 * single-field solves above define it (same symbols, same FP64 phases and
 * exponents).  (These are the plan / launch / destroy calls of a batched
 * interface under the names create / run / destroy, plus status, info,
 * plan, tune and describe.)
 *
 * Radix plans: in FP32 the row tiles of each log2 nx and the column tiles of
 * each log2 ny (a "class") run one of two compiled plans: 0 = stages of
 * radix up to 8 (default), 1 = up to 16.  Both compute the same transforms;
 * results differ by rounding only.  FP64 batches have plan 0 only.
 *
 * fftpde_job: op = FFTPDE_POISSON (coef, t unused), FFTPDE_DIFFUSION
 *   (coef = kappa >= 0, t >= 0) or FFTPDE_WAVE (coef = c >= 0, t finite,
 *   initial velocity 0); nx, ny powers of two in [16, 4096]; lx, ly > 0;
 *   in, out: device fields of nx*ny points (in == out allowed).  No job's
 *   out may overlap another job's in or out.
 * fftpde_batch_create: checks every job, builds the queue (largest jobs
 *   first) in device memory owned by the batch, and captures the launch in a
 *   HIP graph.  The job pointers are fixed here: a run reads the inputs and
 *   writes the outputs the jobs named, so new data is written into the same
 *   buffers between runs.  Errors: EINVAL (any bad job or overlap; nothing is
 *   allocated), ENOMEM, EDEVICE.
 * fftpde_batch_run: enqueues one run on `stream`: replays the captured graph
 *   (use_graph != 0) or launches the same two kernels directly (use_graph = 0,
 *   e.g. inside a caller's own capture).  Runs of one batch share its queue
 *   and counters: runs on different streams must not overlap in time.
 * fftpde_batch_status: waits for `stream`, then returns FFTPDE_OK, or
 *   FFTPDE_ETIMEOUT if a tile's wait for its job's previous step gave up
 *   (about a second; results of that run are then invalid).
 * fftpde_batch_info: number of items in the queue, workgroups launched and
 *   algorithmic HBM bytes of one run (6 field passes per three-pass job, 2
 *   per single-pass job); NULL outputs are skipped.
 * fftpde_batch_plan: sets the radix plan (0 or 1) of one class: kind 0 =
 *   row tiles of log2 length `logn`, 1 = column tiles; logn in [4, 12].
 *   Applies to later runs, graph replays included (the plan is written into
 *   the queue's items in device memory).  Synchronous; the caller ensures
 *   no run of the batch is in flight.  EINVAL for a bad class or plan (plan
 *   1 on an FP64 batch).
 * fftpde_batch_tune: times the batch (graph replays on `stream`, the best of
 *   three groups of `reps` runs; reps < 1: 10) on the data its inputs hold,
 *   then (FP32) flips the plan of each class present, most tiles first, and
 *   keeps a flip if every job's output stays within a relative L2 distance
 *   of 4e-6 * log2(max side) of the starting plan's output and the run got
 *   faster.  Overwrites the outputs; allocates (and
 *   frees) one copy of all outputs.  EINVAL for a batch with a job in place
 *   (its input would change between runs); ETIMEOUT if a run's wait gave up
 *   (the plan of the class then under test is restored).
 * fftpde_batch_describe: a JSON object: dtype, jobs, items, grid, bytes,
 *   single_pass {jobs, items}, classes [{kind "row"|"col", logn, tiles,
 *   plan, max_radix}] and tune [{kind "start"|"row"|"col", logn, plan, us,
 *   err, ok, kept}] (the last tuning's candidates, empty before one).
 *   Writes at most cap bytes (NUL included) to buf (may be NULL); *need
 *   (may be NULL) receives the full length + 1.  EINVAL if it was cut short.
 * fftpde_batch_destroy: frees the batch (waits for nothing: the caller
 *   ensures no run is still in flight); NULL ok. */
typedef struct fftpde_job {
  int op;
  int nx, ny;
  double lx, ly;
  double coef;
  double t;
  const void *in;
  void *out;
} fftpde_job;

int fftpde_batch_create(fftpde_ctx *ctx, const fftpde_job *jobs, int njobs, int dtype,
                        fftpde_batch **batch);
int fftpde_batch_run(fftpde_batch *batch, int use_graph, fftpde_stream stream);
int fftpde_batch_status(fftpde_batch *batch, fftpde_stream stream);
int fftpde_batch_info(const fftpde_batch *batch, long long *items, int *grid, double *bytes);
int fftpde_batch_plan(fftpde_batch *batch, int kind, int logn, int plan);
int fftpde_batch_tune(fftpde_batch *batch, int reps, fftpde_stream stream);
int fftpde_batch_describe(const fftpde_batch *batch, char *buf, size_t cap, size_t *need);
int fftpde_batch_destroy(fftpde_batch *batch);

/* ---- request server ------------------------------------------------------
 * A server runs submitted solves and time evolutions on one GPU with
 * continuous batching: a host thread repeatedly admits queued requests
 * (first come, first served) while the HBM budget and the slots allow, then
 * runs one iteration over the running requests -- each gets its next piece of
 * work (the whole Poisson solve; the forward transforms of an evolution; up
 * to 16 steps of diagnostics; the final field) -- on one of a few streams, so
 * requests overlap on the device and new requests join at the next
 * iteration.  An evolving request keeps the spectra of its initial data on
 * the device between steps (Eq. (solCalorFourier); Eq. (OmegaNonZero),
 * (OmegaZero) with s = 0): a step is the closed form at the absolute time
 * t_n = n dt.  At most two iterations are in flight.
 *
 * fftpde_request: op = FFTPDE_POISSON (steps must be 1), FFTPDE_DIFFUSION
 *   (coef = kappa >= 0, dt >= 0) or FFTPDE_WAVE (coef = c >= 0, dt finite);
 *   dtype; nx, ny powers of two in [2, 4096]; lx, ly > 0; steps >= 1.
 *   in: device field (source s, or u0); v0: wave initial velocity or NULL.
 *   out: device field that receives u at t = steps*dt (Poisson: the
 *   solution), or NULL: the server then owns the output (charged to the
 *   budget) until fftpde_server_release.  diag: NULL, or a device array of
 *   3*steps doubles that receives (mean re, mean im, energy) at t_1..t_steps
 *   (as fftpde_evolve_step); Poisson requests take no diag.  deadline: seconds
 *   after submission (<= 0: none); a request not done by then ends with
 *   FFTPDE_ETIMEOUT.  flags: FFTPDE_REQ_AUTORELEASE forgets the request (and
 *   frees a server-owned output) as soon as it ends, for callers that only
 *   want the statistics.  stream: the request's work starts after the work
 *   enqueued on this stream before submission (e.g. what produced `in`);
 *   NULL: the inputs are ready at submission.  The caller keeps in, v0, out
 *   and diag valid until the request has ended.
 * Budget.  A request is charged its footprint while it runs: the bytes of its
 *   fields (in, v0, out) plus what the server allocates for it (the resident
 *   spectra of an evolution, a reduction scratch, a Poisson solve's spectrum
 *   between its passes, a server-owned output) from a pool of `hbm_budget`
 *   bytes reserved at creation; no request allocates outside the pool.  A request whose footprint
 *   exceeds the whole budget is rejected at submission (FFTPDE_EBUDGET); one
 *   that does not fit now waits, and so do all requests behind it.
 * fftpde_server_create: ctx names the device (the server keeps its own
 *   context and streams); max_slots >= 1 requests run at once; nstreams in
 *   [1, 8].
 * fftpde_server_create_host: the same scheduler with a host backend for
 *   testing it without a GPU: two worker threads stand for the streams, and
 *   every piece of work calls exec(user, id, req, out, phase, n0, nt) on the
 *   request's worker, in order (phase 0: start; 1: steps n0..n0+nt-1; 2: the
 *   final field into out, host memory); a nonzero return fails the request
 *   and skips its remaining work.  The pool is host memory (budget <= 1 GiB).
 * fftpde_server_submit: checks the request (EINVAL, EBUDGET) and queues it;
 *   *id identifies it until released.
 * fftpde_server_poll: FFTPDE_PENDING while queued or running, else the final
 *   status (OK, EDEVICE, ECANCELED, ETIMEOUT, or the host backend's error);
 *   fills *res when res != NULL.  ENOTFOUND for unknown or released ids.
 * fftpde_server_wait: as poll, blocking up to timeout seconds (< 0: forever).
 * fftpde_server_cancel: a queued request ends at once with ECANCELED; a
 *   running one issues no further work and ends with ECANCELED once its work
 *   in flight is done; an ended one is left as it is.
 * fftpde_server_copy_out: enqueues a copy of a successfully ended request's
 *   output (nx*ny points) to dst (device memory, or host memory for the host
 *   backend) on `stream`; EINVAL unless the request ended with FFTPDE_OK.
 * fftpde_server_release: forgets an ended request and frees a server-owned
 *   output; EINVAL if it has not ended.
 * fftpde_server_stats: counters, HBM in use and high-water mark, and the
 *   p50/p99 latency (end - submission, ms) over requests completed OK since
 *   the last reset (reset != 0 resets the latency record and the high-water
 *   mark after reading).
 * fftpde_server_destroy: cancels queued requests, waits for running ones,
 *   stops the thread and frees everything; NULL ok. */
#define FFTPDE_REQ_AUTORELEASE 1

typedef struct fftpde_request {
  int op;
  int dtype;
  int nx, ny;
  double lx, ly;
  double coef;
  double dt;
  long long steps;
  const void *in;
  const void *v0;
  void *out;
  double *diag;
  double deadline;
  int flags;
  fftpde_stream stream;
} fftpde_request;

typedef struct fftpde_result {
  int status;               /* FFTPDE_PENDING, or the final status */
  int state;                /* 0 queued, 1 running, 2 ended */
  double t_submit;          /* seconds on the server clock */
  double t_admit;           /* -1 until admitted */
  double t_done;            /* -1 until ended */
  void *out;                /* where u is (the request's out, or server-owned) */
  long long footprint;      /* bytes charged to the budget */
} fftpde_result;

typedef struct fftpde_stats {
  long long submitted, rejected, admitted, completed, failed, canceled, timed_out;
  long long queued, running;
  long long hbm_budget, hbm_in_use, hbm_high_water;
  long long iterations;
  long long latency_count;  /* completions behind p50 / p99 */
  double p50_ms, p99_ms, mean_ms, max_ms;
  double now;               /* server clock, seconds */
} fftpde_stats;

typedef int (*fftpde_host_exec)(void *user, unsigned long long id, const fftpde_request *req, void *out,
                                int phase, long long n0, int nt);

int fftpde_server_create(fftpde_ctx *ctx, long long hbm_budget, int max_slots, int nstreams,
                         fftpde_server **server);
int fftpde_server_create_host(long long hbm_budget, int max_slots, fftpde_host_exec exec, void *user,
                              fftpde_server **server);
int fftpde_server_submit(fftpde_server *server, const fftpde_request *req, unsigned long long *id);
int fftpde_server_poll(fftpde_server *server, unsigned long long id, fftpde_result *res);
int fftpde_server_wait(fftpde_server *server, unsigned long long id, double timeout, fftpde_result *res);
int fftpde_server_cancel(fftpde_server *server, unsigned long long id);
int fftpde_server_copy_out(fftpde_server *server, unsigned long long id, void *dst, fftpde_stream stream);
int fftpde_server_release(fftpde_server *server, unsigned long long id);
int fftpde_server_stats(fftpde_server *server, int reset, fftpde_stats *stats);
int fftpde_server_destroy(fftpde_server *server);

#ifdef __cplusplus
}
#endif
#endif /* FFTPDE_H */
