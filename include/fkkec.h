/*
 * fkkec.h -- C ABI of the MI355X (gfx950) implementation of fKK-EC:
 * factorized Kramers-Kronig and error correction for CARS hyperspectral
 * images (C. H. Camp Jr., J. S. Bender, Y. J. Lee, arXiv 2005.07132).
 *
 * Orientation (Sec. 2.2): a spectral matrix has M rows (spectra, pixels) and
 * N columns (wavenumbers).  Matrices are row-major; "ld" is the distance in
 * elements between the starts of consecutive rows (ld >= N).
 *
 * Memory: pointers named d_* are device pointers on the context's device,
 * h_* are host pointers.  The caller owns every buffer it passes and keeps it
 * alive until the call's work has finished on the context's stream.  The
 * library owns only what it returns (contexts, bases, servers).  Device
 * scratch of fkk_fit, fkk_plain and fkk_transform comes from the caller when
 * it passes a workspace (d_ws, ws_bytes; fkk_workspace_size gives the size):
 * such a call allocates no device memory except the basis fkk_fit returns.
 * With d_ws NULL (ws_bytes 0) the context uses a workspace of its own, grown
 * on demand and kept until the context is destroyed; the stage calls
 * (fkk_gram, fkk_project, fkk_basis_residual) always use that one.
 *
 * Errors: every call returns an fkk_status; no exception crosses the ABI.
 * Arguments are checked before any launch.  fkk_ctx_last_error() returns a
 * text description of the last failure on that context.
 *
 * Threads: a context is used by one host thread at a time.  A basis is
 * immutable after creation and may be used by several contexts on the same
 * device.
 */
#ifndef FKKEC_H
#define FKKEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FKK_API_VERSION 1

typedef struct fkk_ctx fkk_ctx;
typedef struct fkk_basis fkk_basis;

typedef enum {
    FKK_OK = 0,
    FKK_EINVAL = -1,     /* bad argument (NULL, size, range)                */
    FKK_ENOMEM = -2,     /* device or host allocation failed                */
    FKK_EDEVICE = -3,    /* a HIP call failed                                */
    FKK_EDOMAIN = -4,    /* invalid intensities while strict mode is on      */
    FKK_EMISMATCH = -5,  /* basis and data disagree (N, device)              */
    FKK_ERANK = -7,      /* the requested rank is not available              */
    FKK_EINTERNAL = -8,  /* numerical failure inside the library             */
    FKK_EBUSY = -9       /* not finished within the requested time           */
} fkk_status;

/* Detrending operator D of PEC (Sec. 2.1, Eq. 12, 16). */
enum { FKK_DETREND_ALS = 0, FKK_DETREND_WHITTAKER = 1 };
/* Trendline operator M of SEC (Eq. 4, Eq. 22). */
enum { FKK_SEC_SAVGOL = 0, FKK_SEC_MEAN = 1 };
/* Form of SEC in the conventional method: subtract M{.} of the log
 * magnitude (Eq. 19, as fSEC does on the basis) or divide K' = K e^{H{phi_err}}
 * e^{-i phi_err} by M{Re K'} (Eq. 4-5).  fkk_fit takes the log form only. */
enum { FKK_SEC_FORM_LOG = 0, FKK_SEC_FORM_RE = 1 };
/* Padding of the discrete Hilbert transform. */
enum { FKK_PAD_EDGE = 0, FKK_PAD_ZERO = 1 };
/* Variance scaling f(w) of Eq. 9-10. */
enum { FKK_F_ONE = 0, FKK_F_NOISE = 1 };
/* Which plane of K_CARS (Eq. 23) the output holds. */
enum { FKK_OUT_IM = 0, FKK_OUT_RE = 1, FKK_OUT_ABS = 2 };
/* Precision of the matrix-core contractions.  FP32 and BF16 accumulate in
 * FP32.  The FP32 Gram sums each 32-row stage in FP32 and the stages in FP64;
 * the BF16 Gram sums a whole row chunk (about M / 64 rows) in FP32 and the
 * chunks in FP64.  BF16 rounds the operands (log ratio, projection weights, Z
 * and the corrected bases) to BF16, nearest even, as they are staged.  FP64 (Gram only) promotes the
 * FP32 log ratio to FP64 and accumulates in FP64 on the FP64 matrix cores:
 * the tail of the Gram's spectrum (eigenvalue gaps of ~1e-9 of the largest
 * on tissue cubes) then moves the retained subspace, and with it the
 * sub-sampled rows of Eq. 13-15, only by the FP32 rounding of the log ratio.
 * SPLIT as gram_prec reaches FP64 accuracy on the int8 matrix cores: the log
 * ratio is computed in FP64, scaled per column by a power of two and cut
 * into four int8 slices (an error-free splitting, Ozaki et al. 2012, of 27
 * bits below the column's largest |l|), the slice products of levels up to
 * 2^-21 are summed exactly in int32 and recombined exactly in FP64 per row
 * chunk, and the chunks summed in FP64: the Gram then differs from the
 * exact Gram of the FP64 log ratio by at most about 2^-27 of the columns'
 * largest entries per product, below the FP32 rounding of the log ratio
 * that the FP64 mode keeps.  The column exponents come from every 16th
 * row with one bit of headroom; if a row does not fit, the pass is redone
 * with exact exponents (the result is the same to the bound above).
 * SPLIT as recon_prec reaches FP32 accuracy in the fit's projection and
 * in the reconstruction of Eq. 23 on the BF16 matrix cores: the log ratio
 * and the projection weights, then Z and the corrected bases, are each cut
 * into three BF16 pieces (x = x1 + x2 + x3 + r, |r| about 2^-24 |x|), and
 * the six piece products of combined order up to two are summed in FP32;
 * stored-basis projections and transforms with such a basis run in FP32.
 * The eigensolve and the basis-vector KK / PEC / SEC are FP64 always. */
enum { FKK_PREC_FP32 = 0, FKK_PREC_BF16 = 1, FKK_PREC_FP64 = 2, FKK_PREC_SPLIT = 3 };
/* Route of the truncated SVD (Eq. 6) in fkk_fit. */
enum { FKK_SVD_GRAM = 0, FKK_SVD_RANDOMIZED = 1 };

/*
 * Method parameters.  Fill with fkk_params_default() and override fields.
 * Values the paper leaves open take the documented readings:
 *   fft_len 0     -> smallest power of two >= 3N (padding of H)
 *   als_lambda 0  -> 1e5 * (N/1000)^4
 *   sg_window 0   -> largest odd number <= N/2
 */
typedef struct {
    int32_t k;             /* retained singular vectors, 1..N (Sec. 2.2);
                              0 in fkk_fit: those above s_max max(M, N) eps
                              (eps of FP32; Sec. 4.1), at least 1, at most
                              min(N, 128); the basis reports the count    */
    int32_t f_mode;        /* FKK_F_ONE or FKK_F_NOISE (Eq. 9)             */
    double alpha;          /* Poisson multiplier of Eq. 9                  */
    double sigma_g;        /* Gaussian noise std of Eq. 9                  */
    int32_t pad_mode;      /* FKK_PAD_EDGE / FKK_PAD_ZERO                  */
    int32_t fft_len;       /* Hilbert FFT length, 0 = automatic           */
    int32_t detrend;       /* FKK_DETREND_*                                */
    double als_lambda;     /* ALS / Whittaker smoothness, 0 = automatic    */
    double als_p;          /* ALS asymmetry p (weight above the baseline)  */
    int32_t als_iters;     /* ALS solves (fixed count)                     */
    double ridge_rel;      /* Eq. 17: lambda = ridge_rel * max eig(X^T X)  */
    int32_t sec_mode;      /* FKK_SEC_*                                    */
    int32_t sg_window;     /* Savitzky-Golay window (odd), 0 = automatic   */
    int32_t sg_order;      /* Savitzky-Golay polynomial order              */
    double ml_lambda;      /* Eq. 25 ridge weight of the stored basis      */
    double ratio_floor;    /* ratios I/I_ref not above it are clamped;
                              at least 2^-126 (else FKK_EINVAL)            */
    int32_t strict;        /* 1: clamped ratios fail with FKK_EDOMAIN      */
    int32_t gram_prec;     /* FKK_PREC_* of the Gram (Eq. 6), FP64 and SPLIT
                              allowed                                      */
    int32_t recon_prec;    /* FKK_PREC_FP32 / _BF16 / _SPLIT of the
                              projection (Eq. 13) and the reconstruction
                              (Eq. 23); stored in the basis and used by its
                              later transforms                             */
    int32_t output;        /* FKK_OUT_*                                    */
    const int64_t* q_override; /* host, optional: rows used as U_ss       */
    int32_t n_q_override;  /* length of q_override (0 = use Eq. 13-15)    */
    /* SVD of Eq. 6 in fkk_fit: FKK_SVD_GRAM (Gram on the matrix cores and
     * the FP64 eigensolve, exact to rounding) or FKK_SVD_RANDOMIZED (the
     * randomized range finder the paper names as the alternative for very
     * large data, Sec. 5: Halko, Martinsson & Tropp 2011, subspace iteration
     * with rrf_power_iters passes of A^T, A on l = k + rrf_oversample test
     * vectors (l <= min(N, 128)), then the SVD of Q^T A; approximate in the
     * tail of the spectrum).  gram_prec does not apply to it: its products
     * of A are the FP32 projection and FP64-accumulated products of the FP32
     * log ratio.  A of rank below l fails with FKK_ERANK. */
    int32_t svd_mode;
    int32_t sec_form;         /* FKK_SEC_FORM_* (fkk_plain / fkk_plain_f64)   */
    int32_t rrf_oversample;   /* l - k, >= 0                                 */
    int32_t rrf_power_iters;  /* subspace iterations, >= 0                   */
    uint64_t rrf_seed;        /* test matrix when rrf_omega is NULL          */
    const double* rrf_omega;  /* host, optional: N x l test matrix (row-major);
                                 NULL: standard normal numbers from rrf_seed
                                 (SplitMix64, Box-Muller)                    */
    /* fkk_fit, 0..16: the optional sub-sample between the column extrema
     * of Sec. 2.3 (after Eq. 15).  For each column c of Z = A V_k and
     * j = 1..q_between, the row whose Z value lies nearest (FP32, first row on
     * ties) to min_c + (max_c - min_c) j / (q_between + 1) joins q.
     * Ignored when q_override is given. */
    int32_t q_between;
} fkk_params;

/* Per-fit diagnostics (all fields written by fkk_fit when non-NULL). */
typedef struct {
    int64_t clamps;        /* ratios replaced by ratio_floor               */
    int32_t n_q;           /* rows of U_ss used by fPEC                    */
    double ridge_lambda;   /* lambda of Eq. 17 actually used               */
    double ms_gram;        /* log-ratio + Gram + reduction (device)        */
    double ms_eig;         /* FP64 eigensolve (host)                       */
    double ms_project;     /* projection + sub-sampling (device)          */
    double ms_basis;       /* fKK / fPEC / fSEC on the basis (host FP64)   */
    double ms_recon;       /* reconstruction + epilogue (device)           */
    double ms_total;
    /* device time of the three large kernels, from HIP events recorded on
     * the context's stream around each launch */
    double dev_ms_gram;    /* log ratio + Gram kernel                      */
    double dev_ms_project; /* projection + arg-extrema kernel              */
    double dev_ms_recon;   /* reconstruction + epilogue kernel             */
    double dev_ms_tridiag; /* Householder tridiagonalisation (device)      */
    double dev_ms_logratio;/* log-ratio pass (device)                      */
    int32_t tridiag_path;  /* how the tridiagonalisation ran: FKK_TRIDIAG_* */
} fkk_fit_report;

/* fkk_fit_report.tridiag_path: none (randomized SVD), one cooperative launch
 * with the rows resident in LDS, or one launch per column (forced, beyond
 * the resident size, or after a resident wait gave up). */
enum { FKK_TRIDIAG_NONE = 0, FKK_TRIDIAG_RESIDENT = 1, FKK_TRIDIAG_PER_COLUMN = 2 };

/* Host description of a basis set (Sec. 2.6: f, S, V and the corrected
 * bases).  Arrays are row-major FP64. */
typedef struct {
    int32_t N, k;
    const double* i_ref;   /* N      reference spectrum I_ref              */
    const double* f;       /* N      scaling f(w) of the training data     */
    const double* s;       /* k      singular values                       */
    const double* v;       /* N x k  right singular vectors V_k            */
    const double* b_re;    /* k x N  V^T/f + H{Phi_PEC^T} - V_SEC^T        */
    const double* b_im;    /* k x N  H{V^T/f} - Phi_PEC^T                  */
    double ml_lambda;      /* Eq. 25 ridge weight used by fkk_transform    */
    double ratio_floor;    /* at least 2^-126, as in fkk_params            */
} fkk_basis_desc;

int fkk_version(void);
const char* fkk_status_string(fkk_status s);
void fkk_params_default(fkk_params* p);

/* Context: one device and one HIP stream (NULL = the default stream).  The
 * Householder tridiagonalisation of the eigensolve runs as one cooperative
 * launch whose blocks keep the matrix rows in LDS, when the device supports
 * cooperative launches and the rows fit (N up to about 1,700 on 256 CUs).
 * Its waits for data exchanged between blocks give up after
 * FKK_TRIDIAG_SPIN_LIMIT polls (default 2^22); the context then, and for N
 * beyond that size, uses one launch per
 * column, which it records into a HIP graph (kernel nodes only) the first
 * time it meets an order N and replays on its stream.  Environment, read
 * when the context is created: FKK_NO_RESIDENT_TRIDIAG=1 selects the
 * per-column launches, FKK_NO_GRAPHS=1 launches them one by one. */
fkk_status fkk_ctx_create(int device, void* hip_stream, fkk_ctx** out);
void fkk_ctx_destroy(fkk_ctx* ctx);
const char* fkk_ctx_last_error(const fkk_ctx* ctx);
/* Bytes of device workspace the context currently holds (its own
 * workspace; 0 while every call brought one). */
size_t fkk_ctx_workspace_bytes(const fkk_ctx* ctx);

/* Operations whose device scratch a caller can provide. */
enum { FKK_OP_FIT = 0, FKK_OP_TRANSFORM = 1, FKK_OP_PLAIN = 2 };
/*
 * Bytes of device workspace the operation needs for M spectra of N points
 * with parameters p (FKK_OP_TRANSFORM: p may be NULL; it needs none, so 0).
 * FKK_OP_PLAIN covers fkk_plain and fkk_plain_f64; it may also run in less
 * (its spectra then go through in smaller batches, down to 256 rows).  The
 * size does not depend on the device; ctx may be NULL.  FKK_EINVAL for a bad
 * op, size or parameter set.
 */
fkk_status fkk_workspace_size(const fkk_ctx* ctx, int32_t op, int64_t M, int32_t N, const fkk_params* p,
                              size_t* bytes);

/*
 * fKK-EC on a dataset ("training", Fig. 1b; Eq. 6-23).
 * d_I: M x N FP32 intensities I_CARS (device, stride ld).  h_iref: N FP64
 * reference I_ref (host).  Runs the log ratio and Gram on the device, the
 * eigensolve and the basis-vector KK/PEC/SEC in FP64 on the host, then the
 * projection and (if d_out != NULL) the reconstruction of Eq. 23 into d_out
 * (M x N FP32, stride ld_out, plane selected by p->output).  Returns a new
 * basis in *out_basis (may be NULL if the caller does not want it).
 * d_ws: device workspace of at least fkk_workspace_size(FKK_OP_FIT) bytes,
 * 256-byte aligned, or NULL (the context's own).  Synchronous: returns after
 * d_out is written.
 */
fkk_status fkk_fit(fkk_ctx* ctx, const float* d_I, int64_t M, int32_t N, int64_t ld,
                   const double* h_iref, const fkk_params* p, fkk_basis** out_basis,
                   float* d_out, int64_t ld_out, void* d_ws, size_t ws_bytes,
                   fkk_fit_report* rep);

/*
 * ML:fKK-EC (Fig. 1c; Eq. 24-25 then Eq. 23): applies a stored basis to new
 * spectra.  Z_new = A_new V diag(s^2/(s^2+ml_lambda)), out = plane (FKK_OUT_*)
 * of exp(Z B_re + i Z B_im).  d_I: M x basis.N FP32 (stride ld); d_out: M x N
 * FP32 (stride ld_out).
 * d_norms (device, optional, 8-byte aligned): M x 2 FP32, written by the same
 * kernel from the same loads: with A = l diag(f) (the basis's f),
 * d_norms[2m] = ||A_m||^2 and d_norms[2m+1] = ||A_m V||^2 (sums of FP32
 * products; in the BF16 mode from the BF16 projection), so that
 * 1 - sum d_norms[2m+1] / sum d_norms[2m] over any set of rows is the squared
 * relative residual of fkk_basis_residual (the retraining criterion of
 * Sec. 5).  NULL: not computed.
 * The fused kernel keeps Z in LDS and needs no workspace: pass d_ws NULL,
 * ws_bytes 0 (a workspace given is not used).  Asynchronous on the context's
 * stream; no host synchronisation and no allocation.  Each output row depends
 * only on its input row.
 */
fkk_status fkk_transform(fkk_ctx* ctx, const fkk_basis* basis, const float* d_I, int64_t M,
                         int64_t ld, float* d_out, int64_t ld_out, int32_t plane, float* d_norms,
                         void* d_ws, size_t ws_bytes);

/*
 * Conventional per-spectrum KK -> PEC -> SEC (Eq. 2-5, SEC in the log form
 * of Eq. 19) for every row: the comparator of Fig. 1a without the SVD
 * denoising.  Same data conventions as fkk_fit; workspace as in fkk_fit
 * (FKK_OP_PLAIN; a smaller one of at least 256 spectra's share runs the
 * spectra in smaller batches).  Asynchronous.
 */
fkk_status fkk_plain(fkk_ctx* ctx, const float* d_I, int64_t M, int32_t N, int64_t ld,
                     const double* h_iref, const fkk_params* p, float* d_out, int64_t ld_out,
                     void* d_ws, size_t ws_bytes);
/* Same with FP64 intensities in and FP64 K_CARS out (d_I 8-byte aligned);
 * the arithmetic is FP64 in both variants. */
fkk_status fkk_plain_f64(fkk_ctx* ctx, const double* d_I, int64_t M, int32_t N, int64_t ld,
                         const double* h_iref, const fkk_params* p, double* d_out, int64_t ld_out,
                         void* d_ws, size_t ws_bytes);

/* ---- stages of the fit (each step of Fig. 1b on its own) ---------------- */

/*
 * Log ratio and Gram (Eq. 2, Eq. 6): G = l^T l (N x N, FP64, row-major,
 * symmetric) with l = 1/2 ln(I / I_ref) computed in FP32 (rounded to BF16
 * when prec is FKK_PREC_BF16), products summed as FKK_PREC_* describes;
 * plus the column sums of I (FP64, N) and the number of clamped ratios.
 * ratio_floor as in fkk_params (at least 2^-126, else FKK_EINVAL).
 * Synchronous.
 */
fkk_status fkk_gram(fkk_ctx* ctx, const float* d_I, int64_t M, int32_t N, int64_t ld,
                    const double* h_iref, double ratio_floor, int32_t prec, double* h_gram,
                    double* h_colsum, int64_t* h_clamps);

/*
 * Top-k eigenpairs of a symmetric N x N FP64 matrix (host): eigenvalues in
 * descending order, eigenvectors as the columns of h_evecs (N x k row-major),
 * each with its largest-magnitude entry positive.  Householder
 * tridiagonalisation, bisection and inverse iteration.
 */
fkk_status fkk_eigh_topk(const double* h_a, int32_t N, int32_t k, double* h_evals,
                         double* h_evecs);

/*
 * fKK, fPEC and fSEC on the basis vectors (Eq. 7-22) on the host in FP64,
 * given the factors: f (N), s (k), v (N x k), the sub-sampled rows
 * x = Z[q,:] (n_q x k) of Z = U S.  Creates a basis (device copies included).
 */
fkk_status fkk_basis_from_factors(fkk_ctx* ctx, int32_t N, int32_t k, const double* h_iref,
                                  const double* h_f, const double* h_s, const double* h_v,
                                  const double* h_x, int32_t n_q, const fkk_params* p,
                                  fkk_basis** out_basis);

/* Adequacy of a stored basis for new spectra d_I (M x N, device), the
 * retraining criterion of Sec. 5 ("retraining when ... the current basis
 * vectors do not adequately support new data"): with A = l diag(f) (the
 * basis's I_ref and f), the relative residual of the projection onto the
 * basis vectors, ||A - A V V^T||_F / ||A||_F in [0, 1], written to
 * *h_residual (host).  Computed as sqrt(1 - ||A V||^2 / ||A||^2) from the
 * per-spectrum sums of the FP32 projection (FP32), summed in FP64 per block
 * of 128 spectra and over the blocks in a fixed order, so residuals below
 * about 1e-3 are not resolved.  Works in the context's workspace (16 bytes
 * per 128 spectra).  Synchronises the context's stream. */
fkk_status fkk_basis_residual(fkk_ctx* ctx, const fkk_basis* basis, const float* d_I, int64_t M, int64_t ld,
                              double* h_residual);

/* fkk_basis_residual for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result, with the per-block
 * partial sums in a fixed device array of the library
 * (FKK_NOALLOC_MAX_BLOCKS pairs of doubles, about 1 MiB, on every device the
 * library runs on, held until the process ends), so the call allocates
 * nothing.  M up to FKK_NOALLOC_MAX_SPECTRA (FKK_EINVAL beyond, before any
 * launch).  All calls on one device share that array and it keeps the last
 * call's contents: calls that overlap on one device (from several contexts
 * or threads) race, and the caller must serialise them.  Synchronises the
 * context's stream. */
#define FKK_NOALLOC_MAX_BLOCKS 65536
#define FKK_NOALLOC_MAX_SPECTRA (128LL * FKK_NOALLOC_MAX_BLOCKS)
fkk_status fkk_basis_residual_noalloc(fkk_ctx* ctx, const fkk_basis* basis, const float* d_I, int64_t M,
                                      int64_t ld, double* h_residual);

/*
 * Projection and sub-sampling (Eq. 13-15): Z = A V_k = l diag(f) V_k for the
 * rows of d_I (M x N, stride ld) into d_z (M x k FP32, stride ld_z >= k), and
 * the per-column argmax / argmin rows of Z (first row on ties) into h_qmax,
 * h_qmin (k each, host, may be NULL).  Synchronous when h_qmax or h_qmin is
 * given, else asynchronous.
 */
fkk_status fkk_project(fkk_ctx* ctx, const fkk_basis* basis, const float* d_I, int64_t M,
                       int64_t ld, float* d_z, int64_t ld_z, int64_t* h_qmax,
                       int64_t* h_qmin);

/*
 * Reconstruction (Eq. 23): out = plane of exp(Z B_re) exp(i Z B_im) for Z
 * (M x k FP32 device, stride ld_z).  plane: FKK_OUT_*.  Asynchronous.
 */
fkk_status fkk_reconstruct(fkk_ctx* ctx, const fkk_basis* basis, const float* d_z, int64_t M,
                           int64_t ld_z, float* d_out, int64_t ld_out, int32_t plane);

/* ---- basis objects (the stored model of ML:fKK-EC, Sec. 2.6) ------------ */

fkk_status fkk_basis_import(fkk_ctx* ctx, const fkk_basis_desc* desc, fkk_basis** out);
/* Sizes of a basis: N, k and the number of sub-sampled rows used by fPEC. */
fkk_status fkk_basis_info(const fkk_basis* b, int32_t* N, int32_t* k, int32_t* n_q);
/*
 * Copies FP64 host arrays out of a basis; every pointer may be NULL.
 * Sizes: i_ref, f: N; s: k; v: N x k; b_re, b_im, phi_pec_t, v_sec_t, h_v:
 * k x N; q: n_q; scalars: ml_lambda, ratio_floor, ridge_lambda.
 */
fkk_status fkk_basis_export(const fkk_basis* b, double* i_ref, double* f, double* s,
                            double* v, double* b_re, double* b_im, double* phi_pec_t,
                            double* v_sec_t, double* h_v, int64_t* q, double* scalars3);
/* Frees a basis (NULL: nothing).  FKK_EBUSY, and nothing freed, while a
 * server holds it (fkk_server_add_basis until fkk_server_destroy). */
fkk_status fkk_basis_free(fkk_basis* b);
/* Matrix-core precision (FKK_PREC_FP32, _BF16 or _SPLIT) of the projection
 * and reconstruction that fkk_transform, fkk_project, fkk_reconstruct and
 * the server run with this basis (FP32, BF16 and the BF16 pieces are all
 * kept on the device).  Imported bases start in
 * FP32; fitted ones and those made from factors in the params' recon_prec.  Not thread-safe against
 * concurrent transforms with the same basis. */
fkk_status fkk_basis_set_precision(fkk_basis* b, int32_t prec);
fkk_status fkk_basis_get_precision(const fkk_basis* b, int32_t* prec);

/* ---- serving: stored-basis transforms of image tiles as they arrive ------
 *
 * ML:fKK-EC applies a trained basis to new data as it is acquired (Sec. 2.6,
 * "applied to new data as it is acquired").  A server keeps bases resident
 * on one device and processes tiles (any number of spectra) submitted from
 * host memory.  A scheduler thread admits queued tiles while their device
 * bytes fit the HBM budget and an in-flight slot is free, concatenates the
 * admitted tiles of one basis into a single launch (continuous batching:
 * tiles that arrive while others run join the next launch), and overlaps
 * host-to-device copies, the transform and device-to-host copies on separate
 * streams.  Each output row depends only on its input row and the basis, so
 * a tile's result is the same alone or batched with others.
 */
typedef struct fkk_server fkk_server;

typedef struct {
    int64_t hbm_budget_bytes;  /* device bytes for in-flight tiles (in + out) */
    int32_t max_inflight;      /* tiles in flight at once, 1..4096            */
    int64_t max_batch_rows;    /* spectra per launch                          */
    /* Basis adequacy (Sec. 5: retrain when the basis does not support the
     * new data): every tile's relative residual against its basis (as
     * fkk_basis_residual, from the transform's own per-spectrum sums) is
     * returned by fkk_server_wait; a tile whose residual exceeds this
     * threshold is counted as flagged (0: no flagging). */
    double residual_threshold;
} fkk_server_config;

typedef struct {
    int64_t submitted, completed, rejected;
    int64_t spectra;           /* spectra completed                           */
    int64_t launches;          /* transform launches (batches)                */
    double p50_ms, p99_ms, max_ms, mean_ms;  /* submit -> result in host memory */
    double busy_s;             /* wall time from first submit to last completion */
    double mean_batch_tiles;   /* tiles per launch                            */
    int64_t flagged;           /* completed tiles above residual_threshold:
                                  the basis should be refitted (Sec. 5)       */
    double max_residual;       /* largest tile residual seen                  */
} fkk_server_stats;

/* Creates a server on `device` (own streams, own workspace of
 * hbm_budget_bytes, allocated here). */
fkk_status fkk_server_create(int device, const fkk_server_config* cfg, fkk_server** out);
/* Makes a basis resident for this server; *basis_id identifies it in
 * fkk_server_submit.  Its tiles run in the basis's precision at the time of
 * this call.  The server holds the basis until it is destroyed:
 * fkk_basis_free fails with FKK_EBUSY meanwhile. */
fkk_status fkk_server_add_basis(fkk_server* srv, const fkk_basis* basis, int32_t* basis_id);
/* Queues one tile: h_in (rows x N FP32, stride ld) -> h_out (rows x N FP32,
 * stride ld_out), both host memory (page-locked memory overlaps best) that
 * must stay valid until the tile completes.  Returns immediately with a
 * ticket.  Fails with FKK_ENOMEM if the tile alone exceeds the budget. */
fkk_status fkk_server_submit(fkk_server* srv, int32_t basis_id, const float* h_in, int64_t rows, int64_t ld,
                             float* h_out, int64_t ld_out, int64_t* ticket);
/* Waits until the tile has completed (timeout_ms < 0: no limit).  Returns
 * FKK_OK when done, FKK_EBUSY on timeout.  *latency_ms (nullable) receives
 * submit-to-completion time, *residual (nullable) the tile's relative
 * residual against its basis (see residual_threshold). */
fkk_status fkk_server_wait(fkk_server* srv, int64_t ticket, double timeout_ms, double* latency_ms,
                           double* residual);
/* Blocks until every submitted tile has completed. */
fkk_status fkk_server_drain(fkk_server* srv);
fkk_status fkk_server_stats_get(fkk_server* srv, fkk_server_stats* st);
/* Clears the latency record and counters (bases stay resident). */
fkk_status fkk_server_reset_stats(fkk_server* srv);
void fkk_server_destroy(fkk_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* FKKEC_H */
