/*
 * dpx — multi-wavelength diffractive propagation through cascaded dielectric phase layers
 * and its gradient, on AMD Instinct MI355X (gfx950).
 *
 * What the calls compute (paper: "Wavelength-multiplexed massively parallel diffractive
 * optical information storage and image projection", Section 4 "Optical forward model",
 * Eq. 1, 2, 4, 5; problem statement in Section 2 and the Fig. 1 caption):
 *
 *   for every wavelength lambda_w of a design, starting from the input field u_in
 *   (carried over the input gap z_in by the same propagation when the design has one):
 *     for layer l = 0 .. K-1:
 *       u <- u * t_l,   t_l = exp(-2 pi kappa h_l / lambda) exp(+j 2 pi (n - n_m) h_l / lambda)
 *       u <- P_l u      (Rayleigh-Sommerfeld propagation over the gap z[l], Eq. 4/5,
 *                        evaluated by the angular spectrum: zero-pad N -> pad*N, 2-D FFT,
 *                        multiply by H = exp(+j 2 pi z sqrt(q)) where
 *                        q = (n_m/lambda)^2 - fx^2 - fy^2 > 0 and 0 elsewhere,
 *                        inverse FFT, keep the N x N aperture)
 *     intensity I_w = |u|^2 on the central fov x fov window, summed over bin x bin blocks.
 *
 *   loss (per design): L = (1/W) sum_w (1/T^2) sum_p (I_w,p / sum_p I_w,p
 *                                                     - tau_w,p / sum_p tau_w,p)^2
 *   (the paper's MSE-based loss between projected intensity images and their targets, with
 *    both normalised to unit sum; a wavelength whose intensity or target sums to zero
 *    contributes a zero ratio and a zero gradient.)
 *
 *   backward: dL/dh for every height of every layer given dL/dI (hand-written adjoint:
 *   conjugate transfer function, reverse transforms, d t / d h).
 *
 *   Variants of the propagation: a per-gap lateral translation and axial jitter
 *   (dpx_plan_set_misalignment) and the band-limited transfer function (dpx_design.band_limited)
 *   change H only.  Around the path: per-wavelength PSNR (dpx_psnr), one fused Adam step on the
 *   sigmoid-bounded heights (dpx_adam_step), the phase bit-depth quantiser
 *   (dpx_quantize_heights) and rebinding a plan to new wavelengths (dpx_plan_set_wavelengths).
 *
 * The +j sign of the transmission phase is the reading consistent with the exp(+j k r)
 * outgoing wave of Eq. 4 (the printed Eq. 1 carries -j; with kappa = 0 that is the same model
 * with h -> -h).  n_m is the index of the gap medium ("n" of Eq. 4 and n_air of Eq. 1).
 *
 * Conventions shared by every call:
 *   - Lengths are in metres.  Heights h are float32, fields complex64 stored as interleaved
 *     float pairs (re, im), images float32, all row-major with x fastest.
 *   - Buffers are packed over the plan's designs in design order:
 *        h, dl_dh        : sum_d K_d * N_d * N_d floats          ([K][N][N] per design)
 *        u_in            : sum_d N_d * N_d complex (2 floats each) ([N][N] per design)
 *        intensity, target, dl_di : sum_d W_d * T_d * T_d floats  ([W][T][T] per design)
 *        loss            : n_designs doubles
 *     dpx_plan_layout() reports each design's offsets.
 *   - Every data pointer passed to dpx_forward / dpx_loss / dpx_backward is a caller-owned
 *     DEVICE pointer on the current HIP device, 8-byte aligned (16-byte for fields).
 *     The library never frees them and keeps no reference after the call returns
 *     (except the store-mode state described at dpx_backward).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only enqueues work;
 *     results are ready when the stream has reached that point.
 *   - Every call returns a dpx_status; no exception crosses this interface.  On failure
 *     dpx_last_error() gives a message for the calling thread.
 *   - The plan owns all scratch memory (allocated in dpx_plan_create, released in
 *     dpx_plan_destroy).  dpx_forward, dpx_loss and dpx_backward allocate no device memory
 *     (with opts.use_graph the first call per pointer set instantiates a HIP graph, and the
 *     per-pass timers create HIP events: runtime objects, not workspace).
 *   - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef DPX_H
#define DPX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dpx_status {
  DPX_OK = 0,
  DPX_E_ARG = 1,          /* invalid argument: null pointer, bad shape, misaligned buffer */
  DPX_E_UNSUPPORTED = 2,  /* valid but not built or not applicable: transform length pad*N
                             not in the table, a forced column variant not built for it, the
                             grouped schedule asked for where it cannot run, a misalignment or
                             band limit on a path that cannot apply it */
  DPX_E_NOMEM = 3,        /* device allocation failed or exceeds opts.max_workspace_bytes */
  DPX_E_DEVICE = 4,       /* a HIP runtime error (launch failure, earlier async fault) */
  DPX_E_STATE = 5,        /* call order: store-mode backward without a matching forward */
  DPX_E_NONFINITE = 6     /* opts.check_finite: an output holds a NaN or an infinity */
} dpx_status;

/* One independent design (paper Section 2: K layers of N x N features, N_w wavelengths,
 * each paired with one target image on a shared output field of view).  Host memory; the
 * arrays are copied by dpx_plan_create. */
typedef struct dpx_design {
  int32_t n;         /* N: features per side of every layer (even) */
  int32_t layers;    /* K >= 1 */
  int32_t n_wl;      /* W >= 1 wavelengths */
  int32_t fov;       /* F: side of the central output window, F <= N, (N - F) even */
  int32_t bin;       /* b: detector pixel = b x b samples, F % b == 0; T = F / b */
  int32_t pad;       /* transform length M = pad * N; 2 = zero-padded (linear convolution),
                        1 = periodic window */
  double dx;         /* sampling pitch (feature size), metres */
  double n_medium;   /* refractive index of the gaps (1.0 = air) */
  const double* wl;     /* [W] wavelengths, metres */
  const double* n_mat;  /* [W] real refractive index n(lambda) of the layer material */
  const double* kappa;  /* [W] extinction coefficient kappa(lambda), or NULL for 0 */
  const double* z;      /* [K] z[l] = gap after layer l (z[K-1]: last layer -> output plane) */
  double z_in;          /* gap from the input plane (u_in, e.g. the illumination aperture) to
                           layer 1, metres; 0 = u_in is the field at layer 1 (Fig. 1: the input
                           plane, the layers and the output plane are connected by diffraction).
                           A design with z_in > 0 runs the per-design schedule. */
  int32_t band_limited; /* 0: angular spectrum as above; 1: band-limited angular spectrum
                           (Matsushima and Shimobaba): H = 0 where |fx| or |fy| exceeds
                           (n_m / lambda) / sqrt((2 z / (M dx))^2 + 1), the frequency beyond which
                           the sampled transfer function aliases.  Uses the per-element column
                           variants (0, 1) and the per-design schedule; not with transfer tables,
                           the matrix-core variant or lateral translations. */
} dpx_design;

typedef struct dpx_opts {
  int32_t checkpoint_mode;  /* 0: forward stores the field after every transmission
                               ((K-1)*W*N*N complex per design, K*W*N*N with an input gap
                               z_in > 0: without one, the field after the first layer is
                               u_in t_0(h), which the backward rebuilds from u_in and h) for
                               the backward;
                               1: backward recomputes the forward chunk by chunk */
  int32_t wl_chunk;         /* wavelengths per chunk (0 = automatic) */
  int32_t use_graph;        /* nonzero: the first dpx_forward / dpx_loss / dpx_backward with a
                               given set of buffer pointers captures its launches into a HIP
                               graph, later calls with the same pointers replay it (on a
                               plan-owned stream ordered after and before the caller's stream
                               by events).  Buffer contents may change between calls; the
                               pointers may not.  Per-pass timers run the launches directly. */
  int32_t autotune;         /* nonzero: dpx_plan_create times every column-pass variant and
                               radix plan, and the radix plans of the row passes, on each
                               distinct transform length (up to 256 of a design's wavelengths,
                               three interleaved rounds) and keeps the fastest.  With the
                               environment variable DPX_TUNE_CACHE naming a file, the choices
                               are appended there per (length, pad, band limit, timed
                               wavelengths) and later plans, in any process, take them from
                               it without timing. */
  int32_t force_variant;    /* -1: automatic (autotuned if asked, else a built-in choice per
                               transform length); otherwise a column-pass variant index
                               (see dpx_variant_count / dpx_variant_name).  The transform
                               variants (0-3) give the same results bit for bit; variant 4
                               (DFT as complex matrix products on the FP32 matrix cores,
                               transform lengths up to 512) agrees with them to rounding.
                               DPX_E_UNSUPPORTED if the variant is not built for a design. */
  int32_t transfer_table;   /* transfer function H(|kx|, |ky|) / M^2 of every wavelength and
                               distinct gap precomputed at plan creation ((M/2+1)^2 complex
                               values per wavelength and gap) and read by the column passes:
                               0 = automatic (currently never: on MI355X the table reads
                               cost the column pass more than the evaluation they replace),
                               1 = never (evaluated in the column pass), 2 = always.
                               The table holds the values the column pass would evaluate, so
                               results are bitwise identical either way. */
  int64_t max_workspace_bytes; /* 0 = no limit; otherwise plan creation fails with
                                  DPX_E_NOMEM if the plan would need more */
  int32_t streams;          /* wavelength chunks processed concurrently on this many streams
                               (the caller's plus streams the plan owns); 0 = automatic (1).
                               Several designs in one plan run side by side on up to 4
                               streams (or `streams`, if > 1); 1 keeps everything on the
                               caller's stream.
                               The dL/dh summation order follows the lane layout, so results
                               agree to rounding across settings and bit for bit per setting. */
  int32_t schedule;         /* how the passes of several designs are launched:
                               0 = automatic (grouped when the plan holds several designs, no
                               more than one stream is asked for and the grouped schedule
                               applies; otherwise per design);
                               1 = one launch per design and pass (designs on `streams`);
                               2 = grouped: each pass of all designs that share a transform
                               length, pad and mode is one launch (at most 64 designs per
                               launch), in the order of the layers; the designs are split
                               longest-first into up to 4 partitions (`streams` if > 1, one
                               if `streams` is 1) whose launch lists run side by side on their
                               own streams.  Needs checkpoint_mode 0,
                               every design in one wavelength chunk on one stream and a
                               transform column variant (0-3), else DPX_E_UNSUPPORTED.
                               Results are bitwise identical across schedules. */
  int32_t small_path;       /* 0 = the multi-pass kernels; 1 = for transform lengths up to 128
                               (pad 2; up to 96 with pad 1) in store mode, per-design schedule,
                               one stream, no forced column variant and no transfer tables,
                               each wavelength's plane stays in LDS and the forward (with the
                               binning) and the adjoint (with the dL/dh partials, one slot per
                               wavelength) are one launch each.  Same bits either way.  Not the
                               default: measured on MI355X it ties the multi-pass kernels on
                               a few wavelengths and is slower on many (one block per CU). */
  int32_t check_finite;     /* nonzero (a debugging aid): dpx_forward, dpx_loss and
                               dpx_backward count the NaN and infinite values in what they
                               wrote (intensities; loss and dL/dI; dL/dh), wait for the stream
                               and return DPX_E_NONFINITE naming the output and the count.
                               Such calls synchronise, so they cannot be stream-captured.
                               0: no scan, no synchronisation. */
  int32_t force_plan;       /* radix plan of the transforms (see dpx_radix_plan_count /
                               dpx_radix_plan_name): -1 = automatic (with autotune, the
                               fastest plan of each pass kind is timed and kept per design,
                               else plan 0); k >= 0 = plan k for the row and column passes of
                               every design (DPX_E_UNSUPPORTED where a transform length has no
                               plan k).  Plans other than 0 run the per-design schedule with
                               the evaluated transfer function of untranslated full-spectrum
                               gaps; a column pass that needs another H source (transfer
                               tables, band limit, a lateral translation) runs on plan 0.
                               Different plans agree to rounding, not bit for bit. */
} dpx_opts;

/* Offsets (in elements of the buffer's type) of one design inside the packed buffers. */
typedef struct dpx_layout {
  int64_t h_offset, h_count;       /* floats */
  int64_t u_offset, u_count;       /* complex elements */
  int64_t img_offset, img_count;   /* floats */
  int32_t transform_len;           /* M = pad * N */
  int32_t target_side;             /* T = fov / bin */
  int64_t workspace_bytes;         /* device bytes the plan holds for this design */
  int32_t transfer_tables;         /* transfer tables held for this design (one per distinct
                                      gap; 0 = H is evaluated in the column passes) */
  int32_t lds_path;                /* 1: this design runs LDS-resident (dpx_opts.small_path) */
} dpx_layout;

typedef struct dpx_plan dpx_plan;

/* Fills *opts with the defaults (store mode, automatic chunking, no limit). */
void dpx_opts_default(dpx_opts* opts);

/* Validates the designs, copies their host arrays, builds the per-wavelength constant
 * tables and twiddle tables, and allocates every device buffer the calls need on the
 * current HIP device.  designs: [n_designs] host array; opts may be NULL (defaults).
 * On success *out owns the plan.  Errors: DPX_E_ARG (shape rules above, option ranges),
 * DPX_E_UNSUPPORTED (pad*N not one of 64, 96, 128, 192, 256, 384, 512, 1024, 1600; a forced column
 * variant not built for a design; schedule 2 where it cannot run), DPX_E_NOMEM,
 * DPX_E_DEVICE. */
dpx_status dpx_plan_create(const dpx_design* designs, int32_t n_designs, const dpx_opts* opts,
                           dpx_plan** out);

/* Host-only dry run: validates like dpx_plan_create and reports the device bytes it would
 * allocate, without touching the GPU. */
dpx_status dpx_plan_query(const dpx_design* designs, int32_t n_designs, const dpx_opts* opts,
                          int64_t* workspace_bytes);

/* Releases the plan and its device memory (synchronises the device first). NULL is a no-op. */
dpx_status dpx_plan_destroy(dpx_plan* plan);

/* Radix plans of the transforms of length M: their count (0 for an unsupported length) and a
 * name listing the radices of each stage, e.g. "16x16x4" (empty for an unknown plan; valid
 * until the next call on this thread). */
int32_t dpx_radix_plan_count(int32_t M);
const char* dpx_radix_plan_name(int32_t M, int32_t plan);

/* The radix plans design `design` runs: its row passes and its column passes. */
dpx_status dpx_plan_radix(const dpx_plan* plan, int32_t design, int32_t* row_plan, int32_t* col_plan);

/* Packed-buffer offsets of design `design` (0 <= design < n_designs). */
dpx_status dpx_plan_layout(const dpx_plan* plan, int32_t design, dpx_layout* out);

/* Replaces the wavelengths of design `design` (paper Section 2: Eq. 1's material index and
 * extinction and Eq. 4's transfer-function radius are all per wavelength and are recomputed from
 * these, in double precision on the host).  Minibatch training (Section 4) and sweeps of probe
 * wavelengths reuse one plan and its workspace this way.
 *   wl, n_mat  [n_wl] (host, read, not retained): wavelengths in metres and material indices
 *   kappa      [n_wl] extinction coefficients (host) or NULL for zero
 *   n_wl       must equal the design's wavelength count at creation
 * Layer heights, gaps, grid, field of view and workspace are unchanged.  Blocks the host until
 * the device is idle (queued passes read the old table), then uploads the table and rebuilds
 * any transfer tables.  A store-mode dpx_backward must follow a new dpx_forward.  Errors: DPX_E_ARG for a bad index, a different count or a value that
 * dpx_plan_create would reject (the plan is then unchanged); DPX_E_DEVICE for a failed copy. */
dpx_status dpx_plan_set_wavelengths(dpx_plan* plan, int32_t design, const double* wl,
                                    const double* n_mat, const double* kappa, int32_t n_wl);

/* Misalignment of design `design` (paper Section 2, robustness to lateral and axial
 * displacements and the training against them): gap l (after layer l; the last one ends at the
 * output plane) is lengthened by dz[l] and translates the field it delivers by
 * (shift_x[l], shift_y[l]).  The translation is the factor exp(-j 2 pi (fx sx + fy sy)) on the
 * gap's transfer function, so it costs no extra memory traffic; it is circular over the padded
 * M x M window.  A layer displaced laterally by D_l maps to gap translations D_l - D_(l+1) and an
 * axial displacement to dz_l = Dz_(l+1) - Dz_l, with the output plane fixed (D_K = 0).
 *   dz, shift_x, shift_y  [n_gaps] metres (host, read, not retained), each may be NULL for zeros
 *   n_gaps                must equal the design's layer count
 * Takes effect for calls issued after it returns (the values travel as kernel arguments); a
 * plan with use_graph drops its captured graphs, after waiting for the device.  Forward and
 * backward must see the same misalignment: a store-mode dpx_backward must follow a new
 * dpx_forward (else DPX_E_STATE).  Errors: DPX_E_ARG for a bad index or count, a
 * non-finite value or a negative gap; DPX_E_UNSUPPORTED for a non-zero misalignment on a design
 * that runs the grouped schedule, the LDS-resident path or transfer tables, or a lateral one
 * with the matrix-core column variant or the band-limited spectrum.  On error the plan is
 * unchanged. */
dpx_status dpx_plan_set_misalignment(dpx_plan* plan, int32_t design, const double* dz,
                                     const double* shift_x, const double* shift_y, int32_t n_gaps);

/* Phase bit depth (paper Section 2, limited axial resolution of fabricated thicknesses):
 * h_q[i] = k * (h_max / (2^bits - 1)) with k = rint(h[i] * (2^bits - 1) / h_max) (ties to even)
 * clamped to [0, 2^bits - 1]; the level index is decided in single precision with the scale and
 * the step rounded once from double.
 *   h, h_q  [n] f32 (device; h_q may equal h)    h_max > 0 metres    1 <= bits <= 24
 * Training with quantised heights runs the forward and backward on h_q and applies dL/dh_q to
 * the continuous heights (straight-through).  Errors: DPX_E_ARG for bad arguments. */
dpx_status dpx_quantize_heights(const float* h, float* h_q, int64_t n, double h_max, int32_t bits,
                                void* stream);

/* Totals over all designs: h floats, u_in complex elements, image floats. */
dpx_status dpx_plan_sizes(const dpx_plan* plan, int64_t* h_count, int64_t* u_count,
                          int64_t* img_count);

/* Forward pass (Eq. 1, 2, 5 and the output intensity).
 *   h         [sum K N N] heights in metres (device, read)
 *   u_in      [sum N N] complex input fields (device, read) or NULL for unit plane waves
 *   intensity [sum W T T] output images (device, written)
 * In store mode the plan also records the per-layer fields for dpx_backward. */
dpx_status dpx_forward(dpx_plan* plan, const float* h, const float* u_in, float* intensity,
                       void* stream);

/* Loss and its gradient with respect to the intensities (see the header comment).
 *   intensity, target [sum W T T] (device, read);  loss [n_designs] doubles (device, written);
 *   dl_di [sum W T T] (device, written; may be NULL to skip). */
dpx_status dpx_loss(dpx_plan* plan, const float* intensity, const float* target, double* loss,
                    float* dl_di, void* stream);

/* Backward pass: dl_dh = dL/dh given dl_di = dL/dI (Wirtinger adjoint of dpx_forward).
 *   h, u_in as for dpx_forward;  dl_di [sum W T T] (device, read);
 *   dl_dh [sum K N N] (device, written; summed over wavelengths in a fixed order, so the
 *   result is bitwise reproducible).
 * Store mode: needs the most recent dpx_forward on this plan with the same h and u_in
 * pointers, with no dpx_plan_set_wavelengths or dpx_plan_set_misalignment in between, else
 * DPX_E_STATE.  The contents of h and u_in must not change between that forward and this call
 * (the library cannot see a write through the pointers, e.g. by dpx_adam_step: run the
 * forward again after it).  Recompute mode: no precondition. */
dpx_status dpx_backward(dpx_plan* plan, const float* h, const float* u_in, const float* dl_di,
                        float* dl_dh, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, allocation-free
 * serving or training loops, harnesses that forbid hipMalloc): the loss and dL/dI of dpx_loss for
 * the images of ONE design, without a plan.  Same kernels and the same bits as dpx_loss on a plan
 * holding that design.  The per-wavelength partial sums live in a fixed library-owned device
 * array of DPX_STATIC_LOSS_MAX_WL doubles (512 KiB), one per GPU, held until the process ends;
 * the call allocates nothing.  Every call on one GPU shares that array: calls that overlap on
 * one GPU (on different streams, or from different threads) race and may return wrong values.
 *   intensity, target [n_wl][T][T] f32 (device, read);  loss [1] double (device, written);
 *   dl_di [n_wl][T][T] f32 (device, written) or NULL to skip;  1 <= n_wl <= DPX_STATIC_LOSS_MAX_WL.
 * Errors: DPX_E_ARG (NULL or misaligned pointers, n_wl or T out of range; nothing is enqueued),
 * DPX_E_DEVICE (launch failure, a pending device error). */
#define DPX_STATIC_LOSS_MAX_WL 65536
dpx_status dpx_loss_static(const float* intensity, const float* target, int32_t n_wl, int32_t T,
                           double* loss, float* dl_di, void* stream);

/* Per-wavelength PSNR of the intensity images against the targets (evaluation, Section 2:
 * output PSNR per image-wavelength pair), both normalised to unit sum as in the loss:
 *   psnr_w = 10 log10( max_p tau_w,p^2 / mean_p (I_w,p - tau_w,p)^2 )   (normalised images)
 * The paper's peak convention is in its missing supplement; this is the textbook PSNR with the
 * target's peak.  intensity, target [sum W T T] (device, read); psnr [sum W] doubles, designs
 * in order (device, written; +inf where the images agree exactly). */
dpx_status dpx_psnr(dpx_plan* plan, const float* intensity, const float* target, double* psnr,
                    void* stream);

/* One optimizer step for training the heights (Section 4: Adam with the optimizer library's
 * defaults b1 = 0.9, b2 = 0.999, eps = 1e-8 and learning rate 0.001).  The heights are bounded
 * to [0, h_max] through an unconstrained variable, h = h_max sigmoid(theta); given
 * dl_dh = dL/dh (dpx_backward) the step updates, for each of the n elements,
 *   g = dl_dh h_max s (1 - s)   (s = sigmoid(theta)),
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   theta -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps),
 *   h = h_max sigmoid(theta).
 * theta, h, m, v [n] (device, read and written; m and v start at 0), dl_dh [n] (device, read);
 * step counts from 1.  Single precision; the bias corrections are formed in double. */
dpx_status dpx_adam_step(float* theta, float* h, const float* dl_dh, float* m, float* v, int64_t n,
                         int32_t step, double lr, double b1, double b2, double eps, double h_max,
                         void* stream);

/* Pass kinds reported by the per-pass timers. */
typedef enum dpx_pass {
  DPX_PASS_COL_FWD = 0,       /* column pass with H (forward) */
  DPX_PASS_COL_ADJ = 1,       /* column pass with conj(H) (adjoint) */
  DPX_PASS_ROW_FWD_FIRST = 2, /* u_in * t_0 -> row FFT (no checkpoint: see ROW_ADJ_LAST) */
  DPX_PASS_ROW_FWD_MID = 3,   /* row IFFT -> crop -> * t_l -> row FFT */
  DPX_PASS_ROW_FWD_LAST = 4,  /* row IFFT -> output field of view */
  DPX_PASS_ROW_ADJ_SEED = 5,  /* 2 dL/dI o -> row FFT */
  DPX_PASS_ROW_ADJ_MID = 6,   /* row IFFT -> dL/dh partial -> * conj(t_l) -> row FFT */
  DPX_PASS_ROW_ADJ_LAST = 7,  /* row IFFT -> dL/dh partial (first layer; without an input
                                 gap its field after the transmission, u_in * t_0, is rebuilt
                                 from u_in and h instead of read back) */
  DPX_PASS_LDS_FWD = 8,       /* LDS-resident forward of a whole design (short transforms) */
  DPX_PASS_LDS_ADJ = 9,       /* LDS-resident adjoint of a whole design */
  /* the column launches that read and keep every aperture row (one kernel instance each: all
   * but the last forward and the first adjoint column pass), counted a second time here; they
   * are a subset of DPX_PASS_COL_FWD / DPX_PASS_COL_ADJ */
  DPX_PASS_COL_FWD_FULL = 10,
  DPX_PASS_COL_ADJ_FULL = 11,
  DPX_PASS_COUNT = 12
} dpx_pass;

/* Per-pass timers (measurement support).  While enabled, every launch of the passes above is
 * bracketed by a pair of HIP events recorded on the call's stream, and the launch's
 * algorithmic device-memory traffic (bytes the pass must read and write once) is counted.
 * Enabling or disabling clears the counters. */
dpx_status dpx_timing_enable(dpx_plan* plan, int32_t enable);

/* Waits for the recorded events and returns, for pass `pass`, the summed kernel time in
 * milliseconds, the number of launches, the summed algorithmic bytes and the summed
 * algorithmic floating-point operations (each length-M transform counted as 5 M log2 M, each
 * complex product as 6) since the timers were enabled.  Any output pointer may be NULL. */
dpx_status dpx_timing_read(dpx_plan* plan, int32_t pass, double* total_ms, int64_t* launches,
                           int64_t* bytes, double* flops);

/* Message for the last failed call on this thread ("" if none).  Valid until the next call
 * on this thread. */
const char* dpx_last_error(void);

/* Column-pass kernel variants: count, and a short name for index v ("" if out of range). */
int32_t dpx_variant_count(void);
const char* dpx_variant_name(int32_t v);

/* The column-pass variant the plan uses for design `design`. */
dpx_status dpx_plan_variant(const dpx_plan* plan, int32_t design, int32_t* variant);

/* The schedule the plan runs: 1 = per design, 2 = grouped (see dpx_opts.schedule). */
dpx_status dpx_plan_schedule(const dpx_plan* plan, int32_t* schedule);

/* Library version string. */
const char* dpx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DPX_H */
