/*
 * pact.h -- C ABI of libpact, the MI355X (gfx950) hot path of self-supervised
 * speed-of-sound (SOS) and image joint reconstruction for ring-array
 * photoacoustic computed tomography, after Li, Cui, Ma, Alexander,
 * "Coordinate-based Speed of Sound Recovery for Aberration-Corrected
 * Photoacoustic Computed Tomography" (ICCV 2025).
 *
 * Conventions shared by every call
 * --------------------------------
 * Units: lengths in mm, times in us, SOS in mm/us (1 mm/us = 1000 m/s),
 * sampling rates in samples per us.
 *
 * Grids are centred on the origin: cell (r, c) of an ny x nx grid with
 * spacing s has centre x = (c - (nx-1)/2) s, y = (r - (ny-1)/2) s; arrays are
 * row-major with the row index (y) first.  Element n of the ring sits at
 * R (cos phi_n, sin phi_n), phi_n = phi0 + 2 pi n / n_elem.
 *
 * Complex arrays are interleaved (re, im) float pairs, row-major.  A "full"
 * spectrum of a P x P patch is [P][P] in FFT order (index u carries
 * frequency u or u - P, the usual FFT layout); a "half" spectrum keeps the
 * columns 0 .. P/2 only, [P][P/2 + 1], which is enough for the spectrum of a
 * real patch.  The forward transform is unnormalised with kernel e^{-j k.r};
 * k is the angular wavenumber 2 pi fftfreq(P, px) in rad/mm.
 *
 * Memory: every array pointer is a DEVICE pointer owned by the caller unless
 * the argument says host.  The library allocates no device memory, frees
 * nothing and keeps no pointer after a call returns.  Workspaces are
 * caller-provided; their size comes from the matching *_workspace_size call.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  Every call only enqueues work on that stream and returns; errors
 * raised by a kernel surface at the caller's next synchronisation.  No call
 * synchronises, allocates, or issues a memset, so a sequence of calls can
 * be captured into a HIP graph.
 *
 * Geometry structs (pact_ring, pact_grid, pact_patches) are passed by const
 * pointer to host memory, read during the call only.
 *
 * Errors: every call returns PACT_OK (0) or a negative status; argument
 * checks happen on the host before anything is enqueued, so a failed call
 * has no effect.  pact_last_error() returns a message for the calling
 * thread's last failure.  No C++ exception crosses the ABI.
 *
 * Gradients follow PyTorch's convention for complex numbers:
 * dL/dz = dL/dRe(z) + j dL/dIm(z).  Gradient outputs are overwritten unless a
 * call has an `accumulate` flag.
 */
#ifndef PACT_H
#define PACT_H

#include <stddef.h>

#if defined(__GNUC__) || defined(__clang__)
#define PACT_API __attribute__((visibility("default")))
#else
#define PACT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

#define PACT_OK 0
#define PACT_EINVAL (-1)        /* invalid argument (null pointer, bad size)      */
#define PACT_EHIP (-2)          /* HIP runtime or launch error                     */
#define PACT_EWORKSPACE (-3)    /* workspace missing or smaller than required      */
#define PACT_EUNSUPPORTED (-4)  /* valid but outside the library's limits          */

/* Ring array: n_elem elements on a circle of radius `radius` (mm), element 0 at
 * angle phi0 (rad), counter-clockwise. */
typedef struct {
    int n_elem;
    float radius;
    float phi0;
} pact_ring;

/* A grid of ny x nx cells of size `spacing` (mm) centred on the origin. */
typedef struct {
    int ny;
    int nx;
    float spacing;
} pact_grid;

/* Isoplanatic patches: P x P pixels, origins every `stride` pixels in both
 * directions, Gaussian window of full width at half maximum `fwhm` (mm). */
typedef struct {
    int P;
    int stride;
    float fwhm;
} pact_patches;

/* Thread-local message describing the calling thread's last failure ("" if none). */
PACT_API const char* pact_last_error(void);

/* ABI version (incremented on any incompatible change). */
PACT_API int pact_version(void);

/* ---------------------------------------------------------------------------
 * Geometry helpers (host only, no GPU work)
 * ------------------------------------------------------------------------ */

/* Number of patches along y and x: (ny - P) / stride + 1 and (nx - P) / stride + 1
 * (Supp. S1.4: patch centres on a Cartesian grid).  Patch i = a * npx + b. */
PACT_API int pact_patch_count(const pact_grid* img, const pact_patches* pp, int* npy, int* npx);

/* Patch centres, HOST array [npy * npx][2] of (x, y): the mean of each patch's
 * pixel centres. */
PACT_API int pact_patch_centres(const pact_grid* img, const pact_patches* pp, float* centres_host);

/* ---------------------------------------------------------------------------
 * Once per scan
 * ------------------------------------------------------------------------ */

/* Delay-and-sum stack, Eq. DAS (Sec. 3.1), one image per extra delay (Sec. 3.2):
 *   stack[j][r][c] = sum_n S(t = (|p_rc - r_n| - d[j]) / v0, n)
 * S [n_elem][n_t]: channel n sampled at times t0 + m / fs, read by linear
 * interpolation, zero outside the record.  d [M] extra delays (mm).
 * stack [M][img.ny][img.nx].  Distances and sample positions are computed in
 * FP64, the interpolation and the sum in FP32. */
PACT_API int pact_das_stack(const float* S, int n_t, float fs, float t0, const pact_ring* ring, float v0,
                   const float* d, int M, const pact_grid* img, float* stack, void* stream);

/* Windowed patch spectra (Eq. conv, Sec. 3.3):
 *   Y[i][j] = FFT2(g * stack[j][patch i]),  g[u][v] = exp(-((u-(P-1)/2)^2 + (v-(P-1)/2)^2) px^2 / (2 sigma^2)),
 * sigma = fwhm / (2 sqrt(2 ln 2)), px = img.spacing.  Y is complex,
 * [N][M][P][P/2+1] when half != 0, [N][M][P][P] otherwise, N = npy * npx.
 * P <= 96. */
PACT_API int pact_patch_fft(const float* stack, int M, const pact_grid* img, const pact_patches* pp, int half,
                   float* Y, void* stream);

/* Gaussian-weighted stitching of patch images into the image (Supp. S1.4):
 *   image[y][x] = sum_i x[i][y - y_i][x - x_i] / sum_i g[y - y_i][x - x_i]  where the weight sum > 1e-12,
 *   0 elsewhere,
 * over the patches i covering the pixel (patch i = (a, b) at y_i = a stride, x_i = b stride), g the
 * window of pact_patch_fft.  x [N][P][P] (e.g. the deconvolved patches Re(IFFT2 X_hat)), N = npy * npx;
 * image [img.ny][img.nx] (overwritten).  Deterministic (per-pixel gather, fixed order). */
PACT_API int pact_stitch(const float* patches, int N, const pact_grid* img, const pact_patches* pp, float* image,
                         void* stream);

/* Real part of the normalised inverse 2-D transform of B full P x P spectra:
 * x[b] = Re(IFFT2(X[b])), X complex [B][P][P], x [B][P][P].  Used for the
 * PSF h = Re(IFFT2 H) and the deconvolved patch x_hat = Re(IFFT2 X_hat). P <= 96. */
PACT_API int pact_ifft2_real(const float* X, int B, int P, float* x, void* stream);

/* ---------------------------------------------------------------------------
 * Per optimisation step: SOS -> wavefront -> transfer function -> deconvolution -> loss
 * ------------------------------------------------------------------------ */

/* Wavefront error per (patch, element) ray, Eq. TOF and Eq. wf (Sec. 3.1):
 *   w[i][n] = sum_{s < n_samples} dl (1 - v0 / v(c_i + (s + 1/2) dl u_in)),  dl = L_in / n_samples,
 * u_in the unit vector from centre c_i to element n, L_in the distance at which
 * that ray leaves the box |x|, |y| < (G + 1) spacing / 2 outside which the SOS is
 * v0 (or the element distance, if shorter).  v is the bilinear interpolation
 * of the node grid sos [sosg.ny][sosg.nx] (node centres placed like pixel
 * centres), every node outside the grid being v0 (interpolated pixel grid,
 * Sec. 3.3).  centres [N][2] (x, y) must lie inside that box.  w [N][n_elem].
 * (sosg.ny + 2) * (sosg.nx + 2) * 4 bytes must fit in 160 KiB of LDS.
 * support_radius (mm, >= 0; 0 = none): the user's circular mask of Sec. 3.3,
 * outside which the SOS is the fixed background.  Nodes whose centre lies
 * farther than support_radius (1 + 1e-6) from the origin are taken as v0
 * whatever sos holds there, and only the samples that can touch a node inside
 * are evaluated (those within the radius grown by a cell diagonal; the others
 * add exactly zero).
 * staged (optional, DEVICE, may be NULL): the contrast grid of sos that
 * pact_stage_contrast makes with the same v0 and support_radius.  Every
 * workgroup of the ray kernels holds that grid in LDS; given it, they copy it
 * instead of forming it from sos (same results, bit for bit). */
PACT_API int pact_sos_to_delays(const float* sos, const pact_grid* sosg, float v0, const float* centres, int N,
                       const pact_ring* ring, int n_samples, float support_radius, const float* staged, float* w,
                       void* stream);

/* The contrast grid the ray kernels work on: (sosg.ny + 2) x (sosg.nx + 2)
 * floats, row-major, padded node (r, c) = grid node (r - 1, c - 1) holding
 * sos - v0 where that node lies in the grid and inside the support disc
 * (support_radius as for pact_sos_to_delays; 0 = every node), and 0 on every
 * other node and on the one-node ring around the grid.  staged: DEVICE,
 * pact_staged_contrast_floats() floats (overwritten).  An optimisation step
 * forms it once (pact_sos_adjoint_tv_adam_step writes it for the updated SOS)
 * instead of once per workgroup of each ray kernel. */
PACT_API size_t pact_staged_contrast_floats(const pact_grid* sosg);
PACT_API int pact_stage_contrast(const float* sos, const pact_grid* sosg, float v0, float support_radius,
                                 float* staged, void* stream);

/* Adjoint of pact_sos_to_delays: dL_dsos[a][b] = scale * sum_{i,n} dL_dw[i][n] dw[i][n]/dsos[a][b],
 * with dw/dv = dl v0 / v^2 at every sample spread by the bilinear weights.
 * With support_radius > 0 the nodes outside the support do not enter w, so
 * their gradient is exactly zero (as written).
 * scale: optional DEVICE scalar (NULL = 1).  accumulate != 0 adds to dL_dsos.
 * ws: DEVICE workspace of pact_sos_to_delays_adjoint_workspace_size() bytes,
 * which depends on the current device's CU count: one partial node grid per
 * workgroup (about one per CU) when a band of at least 8 node rows, contrast
 * and accumulator, fits in one CU's LDS (the whole grid in one band up to
 * 141 x 141 nodes); else 0 and ws may be NULL (the tiled form).  Not shared by
 * two calls in flight.  The per-workgroup sums are exact integer sums at a
 * fixed-point scale and are combined in a fixed order, so the result is
 * deterministic; a non-finite SOS node, or one at or below zero, makes the
 * result NaN.  staged (may be NULL) as for pact_sos_to_delays (the tiled form,
 * used where the adjoint workspace size is 0, reads sos only). */
PACT_API size_t pact_sos_to_delays_adjoint_workspace_size(const pact_grid* sosg, int N, const pact_ring* ring);
PACT_API int pact_sos_to_delays_adjoint(const float* sos, const pact_grid* sosg, float v0, const float* centres, int N,
                               const pact_ring* ring, int n_samples, float support_radius, const float* staged,
                               const float* dL_dw, const float* scale, float* dL_dsos, int accumulate, void* ws,
                               size_t ws_bytes, void* stream);

/* Transfer functions, Eq. TF (Sec. 3.1), under the e^{-j k.r} forward transform:
 *   H[i][j](k) = 1/2 (e^{+j|k|(d_j - W_i(th))} + e^{-j|k|(d_j - W_i(th + pi))}),  th = atan2(k_y, k_x),
 * W_i(th) the wavefront of patch i at angle th: the ray from c_i at angle th
 * meets the ring at fractional element index f; W is linear between elements
 * floor(f) and floor(f)+1 (cyclic) of w[i].  H full spectrum [N][M][P][P].
 * h_opt (may be NULL): the PSFs Re(IFFT2 H), [N][M][P][P].  P <= 96. */
PACT_API int pact_delays_to_psf(const float* w, const float* centres, int N, const pact_ring* ring, const float* d, int M,
                       int P, float px, float* H, float* h_opt, void* stream);

/* Adjoint of pact_delays_to_psf (H only): dL_dw [N][n_elem] from dL_dH [N][M][P][P]. */
PACT_API int pact_delays_to_psf_adjoint(const float* w, const float* centres, int N, const pact_ring* ring, const float* d,
                               int M, int P, float px, const float* dL_dH, float* dL_dw, void* stream);

/* Multichannel deconvolution, Eq. fm_fourier and Eq. multi-deconv (Sec. 3.2), with
 * the conjugate transpose and a Tikhonov eps:
 *   X[i](k) = sum_j conj(H[i][j](k)) Y[i][j](k) / (sum_j |H[i][j](k)|^2 + eps).
 * Y, H full spectra [N][M][P][P]; X [N][P][P]. */
PACT_API int pact_multichannel_deconv(const float* Y, const float* H, int N, int M, int P, float eps, float* X,
                             void* stream);

/* Adjoint of pact_multichannel_deconv with respect to H:
 *   dL_dH[i][j] = (conj(g) Y_j - 2 Re(conj(g) X) H_j) / (sum |H|^2 + eps),  g = dL_dX[i]. */
PACT_API int pact_multichannel_deconv_adjoint(const float* Y, const float* H, int N, int M, int P, float eps,
                                     const float* dL_dX, float* dL_dH, void* stream);

/* Data term of Eq. jr for given H and X (modular path):
 *   loss = sum_i sum_k |k| sum_j |Y[i][j](k) - H[i][j](k) X[i](k)|^2  (DEVICE scalar, overwritten),
 * and, if not NULL, its partial derivatives at fixed X and at fixed H:
 *   dL_dH[i][j] = -2 |k| r_ij conj(X_i),   dL_dX[i] = -2 |k| sum_j r_ij conj(H_ij),  r = Y - H X.
 * ws: pact_residual_loss_workspace_size() bytes. */
PACT_API size_t pact_residual_loss_workspace_size(int N, int P);
PACT_API int pact_residual_loss(const float* Y, const float* H, const float* X, int N, int M, int P, float px,
                       float* loss, float* dL_dH, float* dL_dX, void* ws, size_t ws_bytes, void* stream);

/* The fused step: Eq. TF + Eq. multi-deconv + data term of Eq. jr and its
 * gradient with respect to the wavefront table, in one pass over the half
 * spectra Y_half [N][M][P][P/2+1] (the spectra of real patches), without
 * storing any transfer function:
 *   loss  (DEVICE scalar, overwritten; may be NULL, which saves a small second
 *         launch when only the gradient is wanted) = sum over all P x P bins as
 *         in pact_residual_loss with H from w and X the deconvolution of Y by H,
 *   dL_dw [N][n_elem] (overwritten; may be NULL),
 *   X_opt (may be NULL): the deconvolved full spectra [N][P][P].
 * ws: pact_loss_and_grad_workspace_size() bytes (the N patch losses; not shared
 * by two calls in flight).  One workgroup per patch; the patch losses are added
 * in a fixed order and the gradient scatter uses exact integer arithmetic, so
 * the result is deterministic.  M <= 16, P <= 128. */
PACT_API size_t pact_loss_and_grad_workspace_size(int N, int M, int P, int n_elem);
PACT_API int pact_loss_and_grad(const float* Y_half, const float* w, const float* centres, int N, const pact_ring* ring,
                       const float* d, int M, int P, float px, float eps, float* loss, float* dL_dw,
                       float* X_opt, void* ws, size_t ws_bytes, void* stream);

/* The same step from projected spectra.  At a bin k every transfer function of
 * Eq. TF is a cosine of one shifted argument, |k| (d_j - wbar) = phi + delta_j
 * with phi = -|k| wbar and delta_j = |k| d_j, so the delay sums of the closed
 * form need only five step-invariant values per patch and bin,
 *   Pc = sum_j cos(delta_j) Y_j,  Ps = sum_j sin(delta_j) Y_j  (complex),  S = sum_j |Y_j|^2,
 * and two per bin, C2 = sum_j cos(2 delta_j), S2 = sum_j sin(2 delta_j).  The
 * two points where the line through the patch centre along k meets the ring
 * (where Eq. TF reads the wavefront table) do not change between steps either.
 * pact_project_spectra computes all of it once per scan (in FP64, stored in
 * FP32) into T, pact_projected_spectra_floats(N, P) floats; with nb = P (P/2+1)
 * half-spectrum bins (in the order of Y_half) and nv = nb + (P even ? P/2 - 1 : 0)
 * virtual bins (the bins, then the Nyquist-row bins at (-k_x, k_y)):
 *   T[(i*5 + c) * nb + bin],  c = Pc.re, Pc.im, Ps.re, Ps.im, S;
 *   T[(N*5 + c) * nb + bin],  c = C2, S2;
 *   T[(N*5 + 2) * nb + (i*2 + h) * nv + v],  h = 0, 1: the two ring hits of
 *     patch i as fractional element indices in [0, n_elem];
 *   T[(N*5 + 2) * nb + (N*2 + c) * nv + v],  c = |k| / (2 pi) in cycles per
 *     unit length, and |k| times the bin's weight in the half-spectrum sum.
 * centres [N][2] are the patch centres and ring the array, as for
 * pact_loss_and_grad.  pact_loss_and_grad_projected then reads 36 bytes per
 * patch and bin instead of 8 M and needs no ring geometry, and gives what
 * pact_loss_and_grad gives on Y_half (same arguments, workspace and limits; M
 * is the number of delays the spectra were projected with, and centres and
 * ring must be those T was made with). */
PACT_API size_t pact_projected_spectra_floats(int N, int P);
PACT_API int pact_project_spectra(const float* Y_half, int N, int M, int P, float px, const float* d,
                                  const float* centres, const pact_ring* ring, float* T, void* stream);
PACT_API int pact_loss_and_grad_projected(const float* T, const float* w, const float* centres, int N,
                                          const pact_ring* ring, int M, int P, float px, float eps, float* loss,
                                          float* dL_dw, float* X_opt, void* ws, size_t ws_bytes, void* stream);

/* pact_loss_and_grad without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, results and limits as pact_loss_and_grad,
 * bit for bit; the per-patch losses go to a scratch array of 16384 floats that
 * the library keeps in each GPU's memory until the process ends (so N <= 16384,
 * else PACT_EUNSUPPORTED).  The array holds the last call's values, and calls
 * that overlap on one GPU race on it (use one stream, or pact_loss_and_grad with
 * a workspace each).  Allocates nothing. */
PACT_API int pact_loss_and_grad_noalloc(const float* Y_half, const float* w, const float* centres, int N,
                                        const pact_ring* ring, const float* d, int M, int P, float px, float eps,
                                        float* loss, float* dL_dw, float* X_opt, void* stream);

/* Total-variation term of Eq. jr (reading: anisotropic, over node pairs with at
 * least one free node, subgradient sign(0) = 0):
 *   loss += lambda * TV(sos),  grad += lambda * dTV/dsos  (grad over all nodes).
 * mask [G] uint8, nonzero = free node.  loss: DEVICE scalar, added to with one
 * float atomic per workgroup (its last bits may differ between runs; grad does
 * not). */
PACT_API int pact_tv_grad(const float* sos, const unsigned char* mask, const pact_grid* sosg, float lambda, float* grad,
                 float* loss, void* stream);

/* Adam step (Sec. 3.3) on the free nodes of sos (size n), PyTorch's update rule:
 *   t += 1; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 *   sos -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * fixed nodes untouched (mask NULL: every entry is free, as for the neural-field
 * parameter vector).  t: DEVICE int[2], zero-filled before the first step:
 * t[0] counts completed steps (device-side, so that the step can be replayed
 * from a HIP graph), t[1] is an internal arrival counter that every call
 * leaves at zero.  Calls that overlap on the same t race. */
PACT_API int pact_adam_step(float* sos, float* m, float* v, int* t, const unsigned char* mask, int n, const float* grad,
                   float lr, float b1, float b2, float eps, void* stream);

/* TV and Adam in one pass (the last two steps of an optimisation step, Eq. jr and Sec. 3.3):
 *   g = grad + lambda dTV/dsos (TV as in pact_tv_grad, at sos_in),  loss += lambda TV(sos_in) (loss may be NULL),
 *   sos_out = Adam(sos_in, g) on the free nodes (as pact_adam_step), sos_out = sos_in on fixed nodes.
 * grad is read only.  sos_out must be a different buffer from sos_in (every node's TV reads its
 * neighbours' old values); callers alternate two buffers.  m, v [G] and t (DEVICE int[2]) as in
 * pact_adam_step. */
PACT_API int pact_tv_adam_step(const float* sos_in, float* sos_out, float* m, float* v, int* t,
                               const unsigned char* mask, const pact_grid* sosg, const float* grad, float lambda,
                               float* loss, float lr, float b1, float b2, float eps, void* stream);

/* The end of an optimisation step in two launches instead of three: the ray adjoint of dL_dw
 * (pact_sos_to_delays_adjoint, scale 1, same support_radius and workspace), then the sum of its
 * per-workgroup partials fused with TV and Adam (pact_tv_adam_step on that gradient; loss may be
 * NULL).  grad (may be NULL) receives the data term's dL/dsos on the free nodes inside the support
 * (0 on the others, whose partials are not read).  Only for grids that take the whole-grid or banded
 * adjoint (pact_sos_to_delays_adjoint_workspace_size() > 0); else PACT_EUNSUPPORTED.  The same
 * results as the three calls, bit for bit, on the free nodes.  staged_in (may be NULL): the
 * staged contrast grid of sos_in (pact_stage_contrast); staged_out (may be NULL; not staged_in):
 * receives that of sos_out, whole, so that the next step's ray calls need not form it. */
PACT_API int pact_sos_adjoint_tv_adam_step(const float* sos_in, float* sos_out, float* m, float* v, int* t,
                                           const unsigned char* mask, const pact_grid* sosg, float v0,
                                           const float* centres, int N, const pact_ring* ring, int n_samples,
                                           float support_radius, const float* staged_in, float* staged_out,
                                           const float* dL_dw, float lambda, float* loss, float lr, float b1,
                                           float b2, float eps, float* grad, void* ws, size_t ws_bytes,
                                           void* stream);

/* ---- Batched solves: one launch per stage over many scans ----
 *
 * Independent scans (each its own geometry, spectra and SOS grid) advance together: every stage of a
 * pixel-grid step (wavefronts, fused loss, ray adjoint, partial sums + TV + Adam) runs as one launch over
 * all scans, each workgroup taking one scan's block from a table.  Every scan keeps the partition of work it
 * has alone (the same workgroups' rays, lanes per ray, length order, fixed-point scales and partial grids),
 * so its results equal those of pact_sos_to_delays, pact_loss_and_grad_projected and
 * pact_sos_adjoint_tv_adam_step on that scan, bit for bit.
 *
 * pact_batch_scan describes one scan: its geometry and optimiser settings, and the DEVICE buffers of its step
 * as those calls take them.  sos[k] and staged[k] (k = 0, 1) are the two SOS buffers and their staged
 * contrast grids (pact_stage_contrast) that the steps alternate: a step of parity k reads sos[k] and
 * staged[k] and writes sos[1 - k] and staged[1 - k].  grad may be NULL.  partial: the adjoint workspace
 * (pact_sos_to_delays_adjoint_workspace_size() bytes); patch_loss: N floats.  Only grids that take the
 * whole-grid or banded adjoint are accepted (as for pact_sos_adjoint_tv_adam_step). */
typedef struct {
    pact_grid sosg;
    pact_ring ring;
    int N, M, P, n_samples;
    float px, v0, support_radius, eps;
    float lambda, lr, b1, b2, adam_eps;
    const float* centres;
    const float* T;
    float* w;
    float* dL_dw;
    float* patch_loss;
    float* loss;
    float* sos[2];
    float* staged[2];
    float* m;
    float* v;
    int* t;
    const unsigned char* mask;
    float* grad;
    float* partial;
    size_t partial_bytes;
} pact_batch_scan;

/* pact_batch_plan checks the scans, plans every stage of both parities and writes the plan: a HOST buffer of
 * pact_batch_plan_bytes(n_scans) bytes (kernel grids, LDS sizes, where the table is) and a DEVICE table of
 * pact_batch_table_bytes(n_scans) bytes (per-scan launch arguments and block ranges), copied synchronously;
 * both are the caller's and must outlive every step that uses them.  The plan captures the ray tilings
 * pact_rays_autotune chose at that time.  n_scans <= 256.
 * pact_batch_step enqueues one step of every scan (5 launches; with with_loss != 0 also each scan's scalar
 * loss, data term plus lambda TV, as pact_sos_adjoint_tv_adam_step adds it).  It reads only the host plan, so
 * it can be captured in a graph. */
PACT_API size_t pact_batch_plan_bytes(int n_scans);
PACT_API size_t pact_batch_table_bytes(int n_scans);
PACT_API int pact_batch_plan(const pact_batch_scan* scans, int n_scans, void* plan, size_t plan_bytes, void* table,
                             size_t table_bytes, void* stream);
PACT_API int pact_batch_step(const void* plan, int parity, int with_loss, void* stream);

/* pact_batch_step_persistent is SWITCHED OFF: it returns PACT_EUNSUPPORTED and launches nothing (an earlier form
 * of its kernel did not finish on the GPU: one-thread branches around its task queue let the compiler loop the
 * other lanes over the same task; the rewritten kernel has not run on the GPU).  As designed, it enqueues the
 * same step as ONE launch: a workgroup per CU takes tasks (one block of
 * one stage of one scan) from a queue held in the table, in an order where every task comes after the tasks it
 * needs, and starts a task once the stages it reads are complete for its scan (per-scan counters in the table).
 * A scan's stage therefore starts as soon as its own previous stage ends, not when that stage ends for every
 * scan; each block runs the same body on the same block number as in pact_batch_step, so the results are the
 * same, bit for bit.  The kernel returns the counters to zero at its end: steps of one plan must not overlap
 * (enqueue them on one stream, or in one graph).  PACT_EUNSUPPORTED when the scans' largest stage does not
 * leave room in a CU's LDS for the kernel's own few bytes.  A wait that has not ended after about a second
 * gives up (the kernel then ends with wrong results rather than hang); it does not occur while every task's
 * inputs come from earlier tasks of the same queue, which the plan guarantees. */
PACT_API int pact_batch_step_persistent(const void* plan, int parity, int with_loss, void* stream);

/* ---- The paper's neural-field SOS: a sinusoidal network on the SOS-grid nodes (Sec. 3.3) ----
 *
 * v[a][b] = v0 + s (w2 . sin(omega0 (W1 (x_b, y_a) + b1)) + b2) + o on the free nodes (mask != 0),
 * v0 on the others; (x_b, y_a) = node centre (placed like pixel centres, spacing sosg.spacing) divided
 * by mask_radius.  params: DEVICE float vector of 4 hidden + 3 values: W1 [hidden][2] (x, y),
 * b1 [hidden], w2 [hidden], b2, s, o (1027 values at the paper's 256 features).  hidden <= 1024.
 * The node grid then feeds pact_sos_to_delays like the pixel grid. */
PACT_API int pact_siren_sos(const float* params, int hidden, float omega0, const unsigned char* mask,
                            const pact_grid* sosg, float mask_radius, float v0, float* sos, void* stream);

/* Adjoint: dL_dparams (overwritten) = sum over the free nodes of dL_dsos dv/dparams.  ws: DEVICE
 * workspace of pact_siren_sos_adjoint_workspace_size() bytes (one partial per 64 nodes); partials
 * are combined in a fixed order. */
PACT_API size_t pact_siren_sos_adjoint_workspace_size(const pact_grid* sosg, int hidden);
PACT_API int pact_siren_sos_adjoint(const float* params, int hidden, float omega0, const unsigned char* mask,
                                    const pact_grid* sosg, float mask_radius, const float* dL_dsos,
                                    float* dL_dparams, void* ws, size_t ws_bytes, void* stream);

/* ---- Neural-field SOS (coordinate network of Sec. 3.3) queried at every ray sample ----
 *
 * Network (128 frequencies, width 128, 4 hidden layers; other sizes return -4):
 *   gamma(p) = [cos(2 pi B p), sin(2 pi B p)],  B [128][2] (x, y) in cycles per mm,
 *   h_l = relu(W_l h_{l-1} + b_l), l = 1..4,  f = w5 . h_4 + b5,
 *   v(p) = v0 + amp tanh(f(p)) inside the mask disc |p| <= mask_radius, v0 outside.
 * params: DEVICE float vector of pact_nf_param_count() values, row-major blocks
 *   W1 [128][256], b1 [128], W2 [128][128], b2, W3, b3, W4, b4, w5 [128], b5 [1].
 * packed: DEVICE BF16 copy of the weights made by pact_nf_pack (round to nearest
 *   even): W1, W2, W3, W4, W2^T, W3^T, W4^T, w5; pact_nf_packed_count() values.
 * The dense layers run on MFMA with BF16 operands (weights, features, hidden
 * activations and, in the adjoint, pre-activation gradients) and FP32
 * accumulation; biases, the head sum, tanh and the ray sum are FP32. */
PACT_API size_t pact_nf_param_count(int n_freq, int width);
PACT_API size_t pact_nf_packed_count(int n_freq, int width);
PACT_API int pact_nf_pack(const float* params, int n_freq, int width, unsigned short* packed, void* stream);

/* Wavefront errors through the neural field, Eq. wf: the ray from centre c_i
 * to element n is clipped to the mask disc (which must lie inside the ring);
 * its chord [t_a, t_b] is sampled at n_samples midpoints,
 *   w[i][n] = dl sum_s (1 - v0 / v(c_i + (t_a + (s + 1/2) dl) u_in)),  dl = (t_b - t_a) / n_samples,
 * and w = 0 for rays that miss the disc.  w [N][n_elem].
 * act (optional, DEVICE, pact_nf_activation_bytes() bytes, or NULL): the pass also stores every
 * sample's hidden activations (BF16) and head output, for pact_nf_sos_to_delays_adjoint to use
 * instead of recomputing them (1.3 KB per sample, 29 GB for 169 x 512 rays x 256 samples; the last
 * 256 bytes per sample are scratch of the adjoint). */
PACT_API size_t pact_nf_activation_bytes(int N, const pact_ring* ring, int n_samples);
PACT_API int pact_nf_sos_to_delays(const float* B, const float* params, const unsigned short* packed, int n_freq,
                          int width, float amp, float mask_radius, float v0, const float* centres, int N,
                          const pact_ring* ring, int n_samples, float* w, void* act, size_t act_bytes,
                          void* stream);

/* Adjoint: dL_dparams = scale * sum_{i,n} dL_dw[i][n] dw[i][n]/dparams (same layout as params,
 * overwritten), by backpropagation through the network at every sample of every ray with a
 * nonzero dL_dw.  scale: optional DEVICE scalar (NULL = 1).
 * act: the buffer filled by pact_nf_sos_to_delays with the same inputs (the stored activations are read
 * once; the adjoint writes the layer-1 pre-activation gradients into the buffer's tail and reads them
 * back), or NULL (four passes recompute the forward activations; same result).
 * ws: DEVICE workspace of pact_nf_sos_to_delays_adjoint_workspace_size() bytes (one partial gradient
 * per CU of the current device, 16 for the second level of their sum, and two partial W1 gradients per
 * CU); not shared by two calls in flight.  Partial gradients are combined in a fixed order. */
PACT_API size_t pact_nf_sos_to_delays_adjoint_workspace_size(int n_freq, int width);
PACT_API int pact_nf_sos_to_delays_adjoint(const float* B, const float* params, const unsigned short* packed,
                                  int n_freq, int width, float amp, float mask_radius, float v0,
                                  const float* centres, int N, const pact_ring* ring, int n_samples,
                                  const float* dL_dw, const float* scale, float* dL_dparams, void* act,
                                  size_t act_bytes, void* ws, size_t ws_bytes, void* stream);

/* Autotuned ray tilings (for scans of many shapes, e.g. batched solves): times the lanes per ray of
 * pact_sos_to_delays (1, 2, 4, .. 64) on this geometry, with HIP events on `stream`, and keeps the
 * fastest for every later call on this device with the same N, ring element count, n_samples, SOS grid
 * size and support radius (the built-in rule applies otherwise).  The choice changes only how each ray's
 * sum is split, so results move in the last bits.  Synchronises the stream; do not call it while a graph
 * is being captured.  w: DEVICE scratch [N][n_elem] (overwritten).  dL_dw, dL_dsos and ws are not used
 * (the adjoint's work items have a fixed length and need no tuning) and may be NULL.  tiling (HOST, 2
 * ints, or NULL) receives {forward lanes per ray, 0}. */
PACT_API int pact_rays_autotune(const float* sos, const pact_grid* sosg, float v0, const float* centres, int N,
                                const pact_ring* ring, int n_samples, float support_radius, const float* dL_dw,
                                float* w, float* dL_dsos, void* ws, size_t ws_bytes, int* tiling, void* stream);

/* ---- Learned warm start: convolutional SOS initialiser ----
 *
 * Not part of the paper's method, which uses no training data (Sec. 3.3): a convolutional network maps
 * the delay-and-sum stack (Eq. DAS), averaged down to the SOS node grid, to a starting SOS for the
 * optimisation of Eq. jr.  Its training scans are generated by the method's own forward model
 * (Eq. TOF through Eq. wf, then Eq. DAS).
 *
 * Tensors are DEVICE BF16, NHWC: [n][H][W][C], channels contiguous.  Built channel counts (ci, co):
 * (16, 64), (64, 64), (64, 16); others return -4.  Operands are BF16, accumulation and biases FP32, results
 * rounded to the nearest BF16.  Every output is overwritten. */

/* 3 x 3 convolution, stride 1, zero padding 1:
 *   y[n][r][c][o] = act(bias[o] + sum_{ky,kx,i} W[o][ky][kx][i] x[n][r + ky - 1][c + kx - 1][i]),
 * act = relu when relu != 0, then y = 0 where mask <= 0 when mask (same layout as y) is not NULL.
 * packed: the weights as made by pact_conv3x3_pack, pact_conv3x3_packed_count(ci, co) BF16 values.
 * bias: DEVICE float [co] or NULL.  The input gradient of a convolution is this call with the packed
 * adjoint weights (ci and co swapped), no bias, and the ReLU mask of the layer below as mask. */
PACT_API size_t pact_conv3x3_packed_count(int ci, int co);
/* weights: DEVICE float [co][3][3][ci].  packed: [co][K] BF16 with K = 9 ci rounded up to 32,
 * k = (3 ky + kx) ci + i, zero beyond 9 ci.  packed_adjoint (or NULL): the weights of the input
 * gradient, [ci][K'] with K' = 9 co rounded up to 32, k = (3 (2 - ky) + (2 - kx)) co + o. */
PACT_API int pact_conv3x3_pack(const float* weights, int ci, int co, void* packed, void* packed_adjoint,
                               void* stream);
PACT_API int pact_conv3x3_bf16(const void* x, int n, int H, int W, int ci, const void* packed, const float* bias,
                               int co, int relu, const void* mask, void* y, void* stream);

/* Weight and bias gradients of a convolution from its input x [n][H][W][ci] and output gradient
 * g [n][H][W][co]: grad (DEVICE float, co * 9 * ci + co values, overwritten) =
 *   dW[o][ky][kx][i] = sum_{n,r,c} g[n][r][c][o] x[n][r + ky - 1][c + kx - 1][i], then db[o] = sum g[..][o],
 * the layout of the weights followed by the bias.  ws: DEVICE workspace of
 * pact_conv3x3_wgrad_workspace_size() bytes (one partial per workgroup, summed in a fixed order). */
PACT_API size_t pact_conv3x3_wgrad_workspace_size(int n, int H, int W, int ci, int co);
PACT_API int pact_conv3x3_wgrad_bf16(const void* x, const void* g, int n, int H, int W, int ci, int co,
                                     float* grad, void* ws, size_t ws_bytes, void* stream);

/* Resampling between resolutions (H, W even, C a multiple of 8; H, W are the larger grid's):
 *   pool2:           y [n][H/2][W/2][C] = mean of x [n][H][W][C] over 2 x 2 blocks
 *   up2_add:         y [n][H][W][C] = x [n][H/2][W/2][C] at the parent pixel + skip [n][H][W][C]
 *   up2_add_adjoint: g_low [n][H/2][W/2][C] = (sum of g_high over the 2 x 2 children) where mask_low > 0
 *                    (mask_low NULL: everywhere), else 0
 *   pool2_adjoint:   g_high [n][H][W][C] = (g_low at the parent / 4 + skip) where mask > 0, else 0
 *                    (skip, mask may be NULL) */
PACT_API int pact_pool2_bf16(const void* x, int n, int H, int W, int C, void* y, void* stream);
PACT_API int pact_up2_add_bf16(const void* x, const void* skip, int n, int H, int W, int C, void* y, void* stream);
PACT_API int pact_up2_add_adjoint_bf16(const void* g_high, const void* mask_low, int n, int H, int W, int C,
                                       void* g_low, void* stream);
PACT_API int pact_pool2_adjoint_bf16(const void* g_low, const void* skip, const void* mask, int n, int H, int W,
                                     int C, void* g_high, void* stream);

/* Network input from a delay-and-sum stack [M][H][W] (DEVICE float): x [H/f][W/f][C] BF16 with
 * x[r][c][m] = scale * mean of stack[m] over the f x f block (r, c), 0 for m >= M (M <= C, C a multiple of 8). */
PACT_API int pact_warm_input(const float* stack, int M, int H, int W, int factor, float scale, int C, void* x,
                             void* stream);

/* Training loss of the network output z [n][H][W][C] (channel 0 used) against the target
 * t [n][H][W] (DEVICE float) on the free nodes (mask [H][W], DEVICE uint8, 1 = free):
 *   loss = norm * sum_{n, free nodes} (z - t)^2 (DEVICE scalar),  g = d loss / d z [n][H][W][C] BF16
 * (channel 0 = 2 norm (z - t) on free nodes, 0 elsewhere and in every other channel).
 * ws: DEVICE workspace of pact_warm_loss_workspace_size() bytes; the block sums are added in a fixed order. */
PACT_API size_t pact_warm_loss_workspace_size(int n, int H, int W);
PACT_API int pact_warm_loss(const void* z, int n, int H, int W, int C, const float* target,
                            const unsigned char* mask, float norm, float* loss, void* g, void* ws, size_t ws_bytes,
                            void* stream);
/* SOS map from the network output: sos [n][H][W] = v0 + scale * z[..][0] on free nodes, v0 elsewhere. */
PACT_API int pact_warm_sos(const void* z, int n, int H, int W, int C, const unsigned char* mask, float v0,
                           float scale, float* sos, void* stream);

/* Synthetic channel data of a training scan (the stand-in for full-wave data): sources b at
 * sources [n_src][2] (x, y mm) with amplitude amp[b] and width sigma[b] (mm); w [n_src][n_elem]: the
 * wavefront errors of Eq. wf from each source to each element (pact_sos_to_delays with the sources as
 * centres).  Arrival time T = (|r_n - c_b| - w[b][n]) / v0 (Eq. TOF), and
 *   S[n][t] = sum_b amp[b] (1 - u^2) exp(-u^2 / 2) over |u| <= 8,  u = v0 (t0 + t / fs - T) / sigma[b],
 * S [n_elem][n_t] DEVICE float. */
PACT_API int pact_ricker_channels(const float* w, const float* sources, const float* amp, const float* sigma,
                                  int n_src, const pact_ring* ring, float v0, int n_t, float fs, float t0, float* S,
                                  void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PACT_H */
