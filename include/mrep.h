/*
 * mrep.h -- C ABI of libmrep: batched point projection and inversion on
 * B-spline curves through cubic Bezier matrix representations, for AMD
 * Instinct MI355X (gfx950).
 *
 * The operations follow the problem statement and method of Wu & Zou,
 * "Matrix representation and GPU-optimized parallel B-spline computing":
 *   - a degree-p B-spline curve C(t) = sum_i N_{i,p}(t) P_i with a clamped knot
 *     vector (Sec. 4, curve definition and eq. bsplinebasis);
 *   - its decomposition into Bezier pieces in matrix form
 *     Q_q = B_p^{-1} M_{q,p,T} A_{q,p,T} P (Sec. 5.2.1, eqs. bsplinematrix,
 *     Mqpt, decomposition, decomfinal), followed for p >= 4 by a G1,
 *     L2-optimal reduction to cubic and error-controlled splitting to a
 *     tolerance (Sec. 5.2.2), for p <= 2 by degree elevation;
 *   - projection: for each query q the global minimiser
 *     t* = argmin_t |q - C(t)| over the whole domain (Sec. 4, eqs. projection
 *     and projections); inversion is projection of an on-curve point
 *     (Sec. 4, eq. inversion).
 *
 * Conventions
 *   - Every function returns int32_t status: MREP_OK (0) or a negative MREP_E_*
 *     code; mrep_last_error() returns a thread-local message for the last
 *     failure on the calling thread.
 *   - Pointer arguments named dev_* or documented as DEVICE are HIP device
 *     pointers owned by the caller (e.g. torch tensors); the library never
 *     allocates device memory visible to the caller and never frees caller
 *     memory.  HOST pointers are read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued on it and the call returns without waiting;
 *     outputs are valid once the caller synchronises that stream.
 *   - Coordinates are xyz interleaved (AoS, 3 doubles per point).
 *   - Parameters t are in the curve's own knot parameter; the domain of a
 *     clamped curve with n control points is [U[p], U[n]].
 *   - Per-query outcomes are flag bits in flags_out, never call failures.
 */
#ifndef MREP_H
#define MREP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MREP_ABI_VERSION 10

/* status codes */
#define MREP_OK 0
#define MREP_E_INVALID_ARG (-1) /* null pointer, negative size, bad option struct */
#define MREP_E_BAD_DEGREE (-2)  /* degree < 1 or > MREP_MAX_DEGREE, or too few control points */
#define MREP_E_BAD_KNOTS (-3)   /* knot vector not non-decreasing, wrong length, not clamped,
                                   empty domain, interior multiplicity > p, or non-finite */
#define MREP_E_TOL (-4)         /* tol_rel <= 0, or a span needed more than MREP_MAX_PIECES_PER_SPAN pieces */
#define MREP_E_SMALL_BUFFER (-5) /* caller buffer smaller than the size the library reported */
#define MREP_E_HIP (-6)         /* a HIP runtime call failed (message in mrep_last_error) */
#define MREP_E_NO_DEVICE (-7)   /* no gfx950 device available to the calling thread */

/* Curves: degrees 1..MREP_MAX_DEGREE.  Up to MREP_POWER_MAX_DEGREE a span's
 * exact form is kept in power form (Horner in the FP64 polish); above it the
 * power basis has no digits left (its coefficients grow like 3^p), so the span
 * is kept as Bezier points and evaluated by de Casteljau.  The paper's GPU
 * design caps the degree at 31 (one 1024-thread block per basis matrix, Sec. 6
 * discussion and limitations); this library has no block-size cap. */
#define MREP_MAX_DEGREE 32
#define MREP_POWER_MAX_DEGREE 15
/* Surfaces (both directions) and the device span kernel (mrep_span_bezier_curves). */
#define MREP_MAX_SURFACE_DEGREE 15
#define MREP_SPAN_MAX_DEGREE 15
#define MREP_MAX_PIECES_PER_SPAN 4096

/* per-query flag bits */
#define MREP_F_POLISHED 0x1u    /* FP64 Newton on the exact degree-p span decided the answer */
#define MREP_F_NEAR_TIE 0x2u    /* another local minimum lies within the tie margin */
#define MREP_F_ILL_COND 0x4u    /* near-tangent: f'/|C'|^2 < 1e-2 at the minimiser */
#define MREP_F_ENDPOINT 0x8u    /* minimiser within 1e-12 (relative) of an end of the curve's domain */
#define MREP_F_OFFCURVE 0x10u   /* invert only: distance above the curve's tolerance */
#define MREP_F_FULLSCAN 0x20u   /* screen candidate list overflowed; every segment was examined */
#define MREP_F_BAD_ID 0x40u     /* curve_id out of range: outputs are NaN / -1 */
#define MREP_F_NN_FALLBACK 0x80u /* seeded call: curves: the certificate failed and the screened pipeline decided; surfaces: the minimum is not on the seeded patch */

/* screen precisions (mrep_opts.precision) */
#define MREP_PREC_FP64 0 /* exhaustive FP64 examination of every segment (no MFMA screen) */
#define MREP_PREC_FP32 1 /* exhaustive FP32 examination of every segment: 32 samples, FP32 Newton and certified
                            bounds, FP64 polish (no MFMA screen; the FP32 tier of the same path) */
#define MREP_PREC_BF16 3 /* BF16 MFMA screen, FP32 accumulate, FP32 Newton, FP64 polish */

typedef struct mrep_plan mrep_plan; /* host-side decomposition result, owned by the library */
typedef struct mrep_geom mrep_geom; /* device view into a caller-owned buffer (non-owning) */

/* Summary of a plan. */
typedef struct {
    int64_t n_curves;
    int64_t n_spans;       /* non-degenerate knot spans over all curves */
    int64_t n_segments;    /* cubic Bezier pieces over all curves */
    int64_t device_bytes;  /* size of the device buffer mrep_upload needs */
    int32_t max_degree;
    int32_t reserved;
    double tol_rel;
} mrep_plan_info_t;

/* Options of a projection call.  Set struct_size = sizeof(mrep_opts) and start
 * from mrep_opts_default(). */
typedef struct {
    int32_t struct_size;
    int32_t precision;      /* MREP_PREC_* */
    int32_t max_candidates; /* screen candidates kept per query (1..48, default 32); overflow -> full scan */
    int32_t flags;          /* MREP_OPT_* bits */
    double tie_rel;         /* near-tie margin relative to the curve's box diagonal (default 2e-6) */
} mrep_opts;

/* mrep_opts.flags: record HIP events around each stage of the call on its
 * stream; read them back with mrep_last_stage_times. */
#define MREP_OPT_TIME_STAGES 0x1
/* mrep_opts.flags: mrep_project_curves / mrep_invert_curves in BF16 mode run
 * the strategy mrep_tune_curves last chose for the geometry (the screen until
 * then); the workspace must then hold mrep_workspace_bytes with this flag. */
#define MREP_OPT_TUNED 0x2
/* mrep_opts.flags: BF16 mode refines each candidate (query, piece) pair with
 * the paper's path instead of the sampled minimum + Newton: Ferrari roots of
 * E' split the piece into monotonic intervals (Sec. 5.2.3), the elimination
 * criterion keeps intervals where E goes from negative to non-negative (Sec.
 * 5.3, Properties 1-2; both piece ends are always candidates), E is rebased to
 * Bernstein form (Sec. 5.3, b = T a) and Bezier clipping locates its root
 * (Sec. 5.4.1, eq. subdivisionmatrix), in FP64.  The finish (FP64 polish on the
 * exact span) and the full-scan fallback are unchanged. */
#define MREP_OPT_CLIP 0x4
#define MREP_STRATEGY_SCREEN 0  /* BF16 MFMA screen, certified candidates, refine */
#define MREP_STRATEGY_SPHERES 1 /* sphere lists (span clusters where compact), refine every listed piece */
#define MREP_N_BOX_SCHEDULES 6  /* schedules of the sphere-list kernel: s = 3 * persistent + log2(lanes / 4) */
#define MREP_N_STAGES 6 /* most stages any call records (see mrep_last_stage_times) */

/* ---------------------------------------------------------------------- */
/* Decomposition (host, FP64)                                              */
/* ---------------------------------------------------------------------- */

/* Decompose n_curves clamped B-spline curves into cubic Bezier pieces.
 *   degree[n_curves]           HOST  degree p of each curve (1..MREP_MAX_DEGREE)
 *   cp_off[n_curves+1]         HOST  CSR offsets (in points) into cp_xyz
 *   cp_xyz[3*cp_off[n]]        HOST  control points, xyz interleaved
 *   knot_off[n_curves+1]       HOST  CSR offsets into knots; curve c has
 *                                    (#points + p + 1) knots
 *   knots[knot_off[n]]         HOST
 *   tol_rel                    tolerance relative to each curve's control-point
 *                              box diagonal: the same-parameter deviation of
 *                              every cubic piece from the exact curve is at most
 *                              tol_rel * diag (Sec. 5.2.2, tolerance alpha)
 *   n_threads                  host threads to use (<= 0: all available)
 *   out                        receives a new plan; free with mrep_plan_free.
 * Each span's exact Bezier form is Q = B_p^{-1} M A P (Sec. 5.2.1; above
 * MREP_POWER_MAX_DEGREE the same points come from the blossom values
 * P(a^{p-j}, b^j) of the span [a, b], since the power basis in between has no
 * digits left there); p = 3 keeps it, p <= 2 elevates it, p >= 4 reduces it
 * with the G1 conditions and the L2-optimal (delta0, delta1) of Sec. 5.2.2 and
 * splits it at the sample of largest deviation until the tolerance holds.
 * Errors: MREP_E_INVALID_ARG, MREP_E_BAD_DEGREE, MREP_E_BAD_KNOTS, MREP_E_TOL. */
int32_t mrep_decompose_curves(int32_t n_curves, const int32_t* degree, const int64_t* cp_off,
                              const double* cp_xyz, const int64_t* knot_off, const double* knots,
                              double tol_rel, int32_t n_threads, mrep_plan** out);

/* Decompose n_curves clamped RATIONAL B-spline (NURBS) curves,
 * C(t) = sum_i N_i,p(t) w_i P_i / sum_i N_i,p(t) w_i.  The paper's method is
 * stated for non-rational curves (Sec. 6, discussion and limitations; Sec. 7
 * names NURBS as future work); this call carries it over:
 *   - each non-degenerate span's exact form is its homogeneous Bezier points
 *     (w x, w y, w z, w), the blossom of the homogeneous control points; the
 *     FP64 polish evaluates them by de Casteljau and the quotient rule;
 *   - the screen and the refine run on POLYNOMIAL cubic pieces: per span, the
 *     cubic through the span's end points with its end derivatives (the G1
 *     conditions of Sec. 5.2.2 with delta0 = delta1 = 1), split at the sample
 *     of largest deviation until a certified bound of the deviation from the
 *     rational curve (sampled maximum plus a derivative bound of the
 *     homogeneous numerator X - W R) is at most tol_rel * diag.
 * Arguments as mrep_decompose_curves, and
 *   weights[cp_off[n]]  HOST  weight of each control point, positive and finite
 * The returned plan uploads, projects, inverts and evaluates exactly as a
 * non-rational one (mrep_upload, mrep_project_curves, ...); the sphere, NN and
 * clip paths see the polynomial pieces.
 * Errors: as mrep_decompose_curves; MREP_E_INVALID_ARG for null or
 * non-positive weights. */
int32_t mrep_decompose_curves_rational(int32_t n_curves, const int32_t* degree, const int64_t* cp_off,
                                       const double* cp_xyz, const double* weights, const int64_t* knot_off,
                                       const double* knots, double tol_rel, int32_t n_threads, mrep_plan** out);

/* Decompose n_curves clamped polynomial B-spline curves ON THE DEVICE: the
 * same pieces, breakpoints and tables as mrep_decompose_curves followed by
 * mrep_upload, bit for bit (the host and the device run the same arithmetic,
 * compiled without contraction).  Steps, each a set of kernels on `stream`:
 * per curve the validation of mrep_decompose_curves and the box; per knot
 * interval the exact Bezier form Q = B_p^{-1} M A P (Sec. 5.2.1, eqs.
 * decomposition / decomfinal) and a prefix sum that numbers the non-empty
 * spans; then level by level (Sec. 5.2.2, the subdivision figure) the G1 cubic
 * with the L2-optimal (delta0, delta1) from the preloaded Gram matrices (eqs.
 * gram, G1-condition, epsl) and its certified deviation bound for every piece
 * of the level, prefix sums that compact the finished pieces and the pieces
 * to split, and the split of each of those at its sample of largest deviation
 * (eqs. submatrix, subLandR) into the next level; finally one small sort per
 * span puts its pieces in parameter order.  mrep_upload builds the screen
 * tables of the returned plan with kernels, device to device.
 *   n_curves                     > 0
 *   degree[n_curves]       HOST  1 .. MREP_SPAN_MAX_DEGREE (higher degrees and
 *                                rational curves: mrep_decompose_curves*)
 *   cp_off[n_curves+1]     HOST  CSR offsets into cp_xyz (points)
 *   cp_xyz[3*cp_off[n]]    DEVICE control points, xyz interleaved, FP64
 *   knot_off[n_curves+1]   HOST  CSR offsets into knots
 *   knots[knot_off[n]]     DEVICE clamped knot vectors, FP64
 *   tol_rel                as mrep_decompose_curves
 *   stream                 HIP stream (NULL: the default stream)
 *   out                    receives a plan holding device arrays; mrep_plan_info,
 *                          mrep_plan_export (copies to the host), mrep_upload and
 *                          mrep_plan_free work on it as on a host plan.
 * The call allocates its device temporaries and the plan's arrays with
 * hipMalloc (freed on return and by mrep_plan_free) and synchronises the
 * stream between levels (each level's counts size the next).
 * Errors: as mrep_decompose_curves (a curve's validation error names it), and
 * MREP_E_HIP (an allocation or a launch failed), MREP_E_NO_DEVICE. */
int32_t mrep_decompose_curves_device(int32_t n_curves, const int32_t* degree, const int64_t* cp_off,
                                     const double* cp_xyz, const int64_t* knot_off, const double* knots,
                                     double tol_rel, void* stream, mrep_plan** out);

/* Summary of a plan.  Errors: MREP_E_INVALID_ARG. */
int32_t mrep_plan_info(const mrep_plan* plan, mrep_plan_info_t* info);

/* Host copies of the decomposition (each output nullable):
 *   seg_off[n_curves+1]  CSR offsets of each curve's pieces
 *   seg_t[2*n_segments]  (t_a, t_b) of each piece in the curve's parameter
 *   seg_cp[12*n_segments] the piece's 4 cubic control points, xyz interleaved
 *   seg_span[n_segments] index of the knot span the piece lies in (global over the plan)
 * Errors: MREP_E_INVALID_ARG. */
int32_t mrep_plan_export(const mrep_plan* plan, int64_t* seg_off, double* seg_t, double* seg_cp,
                         int32_t* seg_span);

void mrep_plan_free(mrep_plan* plan);

/* Copy a plan's tables into a caller-owned DEVICE buffer of at least
 * info.device_bytes bytes (256-byte aligned), asynchronously on `stream`.
 * The returned view stays valid while the buffer lives; release it with
 * mrep_geom_release (which does not touch the buffer).  The plan may be freed
 * once the stream has passed the copy.
 * Errors: MREP_E_INVALID_ARG, MREP_E_SMALL_BUFFER, MREP_E_HIP, MREP_E_NO_DEVICE. */
int32_t mrep_upload(const mrep_plan* plan, void* dev_buf, int64_t bytes, void* stream, mrep_geom** out);

void mrep_geom_release(mrep_geom* geom);

/* ---------------------------------------------------------------------- */
/* Batched device operations                                              */
/* ---------------------------------------------------------------------- */

int32_t mrep_opts_default(mrep_opts* opts);

/* DEVICE workspace size for a projection / inversion of n queries.
 * Errors: MREP_E_INVALID_ARG. */
int32_t mrep_workspace_bytes(const mrep_geom* geom, int64_t n, const mrep_opts* opts, int64_t* bytes);

/* Project n query points, each onto its own curve (curve_id), returning the
 * global minimiser of eq. projection on the EXACT curve.
 *   curve_id[n]  DEVICE int32
 *   q_xyz[3n]    DEVICE double, xyz interleaved
 *   workspace    DEVICE, >= mrep_workspace_bytes(...) bytes, 256-byte aligned
 *   t_out[n]     DEVICE double   minimising parameter
 *   dist_out[n]  DEVICE double   |q - C(t)|
 *   seg_out[n]   DEVICE int32    0-based index of the cubic piece holding t
 *                                within the curve's piece list (mrep_plan_export)
 *   flags_out[n] DEVICE uint32   MREP_F_* bits
 * Queries may come in any order.  Calls on one stream are ordered; the same
 * workspace must not be used by two calls that may overlap.
 * Limits: n * opts->max_candidates < 2^31 (the candidate-pair counter is
 * 32-bit); larger batches are split by the caller.
 * Errors: MREP_E_INVALID_ARG, MREP_E_SMALL_BUFFER, MREP_E_HIP. */
int32_t mrep_project_curves(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* curve_id,
                            const double* q_xyz, void* workspace, int64_t ws_bytes, double* t_out,
                            double* dist_out, int32_t* seg_out, uint32_t* flags_out, void* stream);

/* Counters a curve projection call leaves in its workspace: counts_out[0] =
 * queries whose candidate list overflowed to the full scan, counts_out[1] =
 * candidate (query, piece) pairs reserved for the refine, counts_out[2] =
 * sphere tests |q - c| - r of the sphere-list strategy (cluster and piece
 * spheres; 0 after a call in the screen strategy).  counts_out holds 3
 * entries.  workspace is the
 * one the call used (mrep_project_curves, mrep_invert_curves,
 * mrep_project_curves_seeded, also with MREP_OPT_TUNED), geom its geometry;
 * the read is ordered after the call on stream and waits for it.
 * Errors: MREP_E_INVALID_ARG, MREP_E_HIP. */
int32_t mrep_workspace_counts(const mrep_geom* geom, const void* workspace, int64_t* counts_out, void* stream);

/* Allocation-free projection, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, outputs, options and answers as
 * mrep_project_curves, without the workspace: the kernels use a fixed scratch
 * array of MREP_NOALLOC_SCRATCH_BYTES (64 MiB) that the library holds on each
 * GPU it runs on until the process ends.  The call itself allocates nothing
 * (no hipMalloc, no library allocation).  The scratch is found once per device
 * with that device current (the first call on it).  Every call on a GPU shares
 * that GPU's scratch and each call clears what it needs, so calls that may
 * overlap on one GPU (two streams, two host threads) race: order them.
 * Errors: MREP_E_SMALL_BUFFER when mrep_workspace_bytes(geom, n, opts) exceeds
 * the scratch (about 500k queries at the default options: split the batch),
 * MREP_E_INVALID_ARG (as mrep_project_curves, and MREP_OPT_TIME_STAGES, whose
 * events would be created), MREP_E_HIP. */
#define MREP_NOALLOC_SCRATCH_BYTES (64ll << 20)
int32_t mrep_project_curves_noalloc(const mrep_geom* geom, const mrep_opts* opts, int64_t n,
                                    const int32_t* curve_id, const double* q_xyz, double* t_out,
                                    double* dist_out, int32_t* seg_out, uint32_t* flags_out, void* stream);

/* Inversion (Sec. 4, eq. inversion): as mrep_project_curves, and additionally
 * sets MREP_F_OFFCURVE where the distance exceeds the curve's tolerance
 * tol_rel * diag (the point is then not on the curve). */
int32_t mrep_invert_curves(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* curve_id,
                           const double* q_xyz, void* workspace, int64_t ws_bytes, double* t_out,
                           double* dist_out, int32_t* seg_out, uint32_t* flags_out, void* stream);

/* Monotonic decomposition (Sec. 5.2.3): for each (query, piece) pair, the
 * roots in (0, 1) of E'(u) (eq. E't), the second derivative of the squared
 * distance D(u) = |C(u) - q|^2 on the cubic piece in its local parameter u;
 * between consecutive roots E = D' is monotonic.  method MREP_ROOTS_FERRARI:
 * Ferrari's method on the quartic (at the degree its coefficients show, each
 * root polished by three Newton steps); MREP_ROOTS_NEWTON: Newton's iteration
 * from 8 uniform starts (at most 20 steps each, converged roots in (0, 1)
 * kept once), the numerical method the paper compares against (Table
 * tab:analytical).  FP64, one thread per pair.
 *   curve_id[n]  DEVICE int32   curve of pair i
 *   piece[n]     DEVICE int32   0-based piece index within that curve (mrep_plan_export)
 *   q_xyz[3n]    DEVICE double  query of pair i
 *   roots_out[4n] DEVICE double roots of pair i, ascending, in roots_out[4i..4i+count)
 *   count_out[n] DEVICE int32   number of roots (0..4); -1 for an out-of-range curve or piece
 * Errors: MREP_E_INVALID_ARG (null pointers with n > 0, n < 0, unknown method), MREP_E_HIP. */
#define MREP_ROOTS_FERRARI 0
#define MREP_ROOTS_NEWTON 1
int32_t mrep_monotonic_split(const mrep_geom* geom, int64_t n, const int32_t* curve_id, const int32_t* piece,
                             const double* q_xyz, int32_t method, double* roots_out, int32_t* count_out,
                             void* stream);

/* Evaluate C_{curve_id[i]}(t[i]) on the exact curve (FP64).  t outside the
 * domain is clamped to it.  curve_id[n], t[n], xyz_out[3n]: DEVICE.
 * Out-of-range ids give NaN.  Errors: MREP_E_INVALID_ARG, MREP_E_HIP. */
int32_t mrep_eval_curves(const mrep_geom* geom, int64_t n, const int32_t* curve_id, const double* t,
                         double* xyz_out, void* stream);

/* Span decomposition on the device (Sec. 5.2.1, eqs. `decomposition` and
 * `decomfinal`): the exact degree-p Bezier form of every knot interval of a
 * batch of clamped B-spline curves, one thread per interval, FP64.  Curve c
 * has n_c = cp_off[c+1] - cp_off[c] control points and n_c - p_c knot
 * intervals [U_q, U_{q+1}], q = p_c .. n_c - 1; the Bezier points of each are
 * the blossom values P(U_q^(p-j), U_{q+1}^(j)), j = 0..p, the same points as
 * B_p^{-1} M A P.
 *
 * mrep_span_layout (HOST only): iv_off[n_curves+1] and pt_off[n_curves+1]
 * receive the offsets of each curve's intervals and of its Bezier points:
 * iv_off[c+1] = iv_off[c] + n_c - p_c, pt_off[c+1] = pt_off[c] + (n_c - p_c)(p_c + 1).
 *   Errors: MREP_E_INVALID_ARG, MREP_E_BAD_DEGREE (degree out of range or
 *   fewer than p + 1 points), MREP_E_BAD_KNOTS (knot count not n_c + p_c + 1).
 *
 * mrep_span_bezier_curves: every pointer DEVICE.  max_degree (1..MREP_SPAN_MAX_DEGREE):
 * at least the largest degree in the batch; it picks the kernel instance, and
 * an interval of a curve of higher degree writes NaN to t_out only.  degree, cp_off, knot_off,
 * cp_xyz, knots: the arrays of mrep_decompose_curves; iv_off, pt_off: the
 * output of mrep_span_layout for the same curves, and n_intervals =
 * iv_off[n_curves].  Interval k of curve c writes its p_c + 1 points (xyz
 * interleaved) to bz_out[3 (pt_off[c] + k (p_c + 1)) ..] and [U_q, U_{q+1}] to
 * t_out[2 (iv_off[c] + k) ..].  A zero-length interval (repeated knot) writes
 * NaN points; an interval whose curve's counts disagree with iv_off / pt_off
 * writes NaN to t_out only.  Knots must be non-decreasing; they are not
 * checked.  Enqueued on stream; nothing is allocated.
 *   Errors: MREP_E_INVALID_ARG (null pointers with n_intervals > 0, negative
 *   counts, max_degree out of range), MREP_E_HIP. */
int32_t mrep_span_layout(int32_t n_curves, const int32_t* degree, const int64_t* cp_off, const int64_t* knot_off,
                         int64_t* iv_off, int64_t* pt_off);
int32_t mrep_span_bezier_curves(int32_t n_curves, int64_t n_intervals, int32_t max_degree, const int32_t* degree,
                                const int64_t* cp_off, const int64_t* knot_off, const int64_t* iv_off, const int64_t* pt_off,
                                const double* cp_xyz, const double* knots, double* bz_out, double* t_out,
                                void* stream);

/* Autotuner (BF16 mode): projects the batch with each strategy (one untimed
 * and two timed runs each, HIP events on `stream`), keeps the faster one for
 * this geometry (used by calls with MREP_OPT_TUNED), and leaves its answers in
 * the outputs.  Both strategies return the certified global minimum; they
 * differ in speed, by how compact the curves are against their boxes.  The
 * sphere strategy is timed in each of the MREP_N_BOX_SCHEDULES schedules of
 * its sphere-list kernel (4, 8 or 16 lanes per query; one workgroup per tile
 * of 32 queries in XCD-aware order, or a persistent grid that takes tiles
 * from one queue per XCD and then from the others'), and the fastest schedule
 * is kept for the geometry too (mrep_curve_schedule); the schedules give
 * identical answers.  workspace: mrep_workspace_bytes with MREP_OPT_TUNED.
 * strategy_out (HOST, nullable): the choice; ms_out (HOST double[2],
 * nullable): per-call times of the screen strategy and of the sphere strategy
 * in its best schedule.  Synchronous.  Errors: as mrep_project_curves. */
int32_t mrep_tune_curves(mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* curve_id,
                         const double* q_xyz, void* workspace, int64_t ws_bytes, double* t_out, double* dist_out,
                         int32_t* seg_out, uint32_t* flags_out, int32_t* strategy_out, double* ms_out, void* stream);

/* Set the strategy of calls with MREP_OPT_TUNED directly (MREP_STRATEGY_*),
 * for a caller that knows its workload.  Errors: MREP_E_INVALID_ARG. */
int32_t mrep_set_curve_strategy(mrep_geom* geom, int32_t strategy);

/* The schedule of the sphere-list kernel for this geometry (used by the sphere
 * strategy and the seeded calls): lanes_out (HOST) 4, 8 or 16 lanes per
 * query, persistent_out (HOST) 1 for the persistent grid over per-XCD tile
 * queues, 0 for one workgroup per tile; ms_out (HOST double
 * [MREP_N_BOX_SCHEDULES], nullable): the per-call times of the sphere
 * strategy in each schedule at the last mrep_tune_curves (index 3 * persistent
 * + log2(lanes / 4); zeros before any tune).  The default is 8 lanes, tile
 * map.  Errors: MREP_E_INVALID_ARG (null or surface geometry, null outputs). */
int32_t mrep_curve_schedule(const mrep_geom* geom, int32_t* lanes_out, int32_t* persistent_out, double* ms_out);

/* Set that schedule directly.  lanes: 4, 8 or 16; persistent: 0 or 1.  The
 * answers do not depend on it.  Errors: MREP_E_INVALID_ARG. */
int32_t mrep_set_curve_schedule(mrep_geom* geom, int32_t lanes, int32_t persistent);

/* Durations in milliseconds of the stages of the last call on the calling
 * thread that set MREP_OPT_TIME_STAGES.  mrep_project_curves / invert: 4
 * stages, [0] grouping, [1] screen (0 in the FP64 and FP32 modes), [2] refine of the
 * candidate (query, piece) pairs (0 in those modes), [3] top-2 + FP64 polish +
 * write, with the full scan of overflowed queries (every query in those modes).
 * mrep_project_curves_seeded (and mrep_project_curves in the sphere
 * strategy): 6 stages, [0] grouping, [1] sphere candidates (the box kernel),
 * [2] network scoring (0 without a network), [3] seed + certificate (0
 * without a network), [4] refine of the listed pairs of the undecided queries,
 * [5] their top-2 + FP64 polish + write and the full scan of overflows.
 * mrep_project_surfaces / invert: 3 stages, [0] grouping + sphere lists,
 * [1] sampled bounds + gate + patch minima, [2] top-2 + FP64 polish + write.
 * mrep_project_surfaces_seeded: 4 stages, [0] grouping + sphere lists +
 * candidates, [1] network scoring, [2] seeded Newton + bounds + gate + patch
 * minima, [3] top-2 + FP64 polish + write.  Waits for
 * that call's events.  n = capacity of ms_out (>= MREP_N_STAGES is always
 * enough).  Returns the number of stages written (> 0).
 * Errors: MREP_E_INVALID_ARG (no timed call yet, n too small), MREP_E_HIP. */
int32_t mrep_last_stage_times(double* ms_out, int32_t n);

/* ---------------------------------------------------------------------- */
/* Surfaces (tensor-product B-splines; the paper's matrix form applied in  */
/* u and in v, Sec. 5.2.1, with the curve reduction of Sec. 5.2.2 applied  */
/* to rows, then columns)                                                  */
/* ---------------------------------------------------------------------- */

/* Decompose n_surf clamped tensor-product B-spline surfaces into bicubic
 * Bezier patches.  Per surface s:
 *   deg_u[s], deg_v[s]          HOST  degrees (1..MREP_MAX_SURFACE_DEGREE)
 *   n_u[s], n_v[s]              HOST  control-net size
 *   cp_off[n_surf+1]            HOST  CSR offsets (in points) into cp_xyz; net u-major: P[i * n_v + j]
 *   cp_xyz                      HOST  double xyz
 *   ku_off / ku, kv_off / kv    HOST  CSR knot vectors (n_u + p + 1 and n_v + q + 1 values, clamped)
 *   tol_rel                     tolerance relative to the net's box diagonal
 * Each non-degenerate span patch becomes B_p^-1 D_u P D_v^T B_q^-T exactly
 * (degrees <= 3 elevated to cubic); a direction of degree >= 4 is reduced to
 * cubic with the G1 L2 curve reduction (rows in u, then columns in v), and a
 * patch whose error bound on a 32 x 32 grid exceeds tol_rel * diag is split
 * (on the exact net) in the direction of larger error at the worst grid line.
 * Errors: as mrep_decompose_curves. */
int32_t mrep_decompose_surfaces(int32_t n_surf, const int32_t* deg_u, const int32_t* deg_v, const int32_t* n_u,
                                const int32_t* n_v, const int64_t* cp_off, const double* cp_xyz,
                                const int64_t* ku_off, const double* ku, const int64_t* kv_off, const double* kv,
                                double tol_rel, int32_t n_threads, mrep_plan** out);

/* HOST copies of a surface plan (any output may be NULL):
 *   patch_off[n_surf+1]   first patch of each surface
 *   patch_uv[P][4]        (u_a, u_b, v_a, v_b) of each patch
 *   patch_cp[P][4][4][3]  bicubic Bezier net (u-major)
 *   patch_span[P]         index of the exact span patch within its surface (u-span major)
 * mrep_plan_info on a surface plan reports surfaces in n_curves, patches in
 * n_segments, span patches in n_spans and reserved = 1.
 * Errors: MREP_E_INVALID_ARG (null or curve plan). */
int32_t mrep_plan_export_surfaces(const mrep_plan* plan, int64_t* patch_off, double* patch_uv, double* patch_cp,
                                  int32_t* patch_span);

/* DEVICE workspace size for a surface projection of n queries.
 * Errors: MREP_E_INVALID_ARG (also for a curve geometry). */
int32_t mrep_surface_workspace_bytes(const mrep_geom* geom, int64_t n, const mrep_opts* opts, int64_t* bytes);

/* Project n query points, each onto its own surface, returning the global
 * minimiser of |q - S(u, v)| over the whole domain of the EXACT surface.
 *   surface_id[n] DEVICE int32;  q_xyz[3n] DEVICE double
 *   uv_out[2n]    DEVICE double  (u, v) of the minimiser
 *   dist_out[n]   DEVICE double  |q - S(u, v)|
 *   patch_out[n]  DEVICE int32   index of the bicubic patch holding (u, v) within the surface
 *                                (half-open rectangles, closed at the domain's far sides)
 *   flags_out[n]  DEVICE uint32  MREP_F_POLISHED (always: FP64 Newton on the exact span
 *                                patch decides), MREP_F_NEAR_TIE, MREP_F_ILL_COND (smallest
 *                                relative curvature of the distance < 1e-2),
 *                                MREP_F_ENDPOINT (on the boundary of the domain),
 *                                MREP_F_FULLSCAN, MREP_F_BAD_ID
 * opts->precision and max_candidates are ignored (candidates come from patch
 * bounding spheres; patches are minimised in FP32 and the answer in FP64).
 * Limits: n < 2^31 / 96.  Errors: MREP_E_INVALID_ARG, MREP_E_SMALL_BUFFER, MREP_E_HIP. */
int32_t mrep_project_surfaces(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* surface_id,
                              const double* q_xyz, void* workspace, int64_t ws_bytes, double* uv_out,
                              double* dist_out, int32_t* patch_out, uint32_t* flags_out, void* stream);

/* Inversion: as mrep_project_surfaces, and MREP_F_OFFCURVE where the distance
 * exceeds the surface's tolerance tol_rel * diag. */
int32_t mrep_invert_surfaces(const mrep_geom* geom, const mrep_opts* opts, int64_t n, const int32_t* surface_id,
                             const double* q_xyz, void* workspace, int64_t ws_bytes, double* uv_out,
                             double* dist_out, int32_t* patch_out, uint32_t* flags_out, void* stream);

/* S_{surface_id[i]}(uv[2i], uv[2i+1]) on the exact surface (FP64), clamped to
 * the domain; DEVICE arrays.  Bad ids give NaN. */
int32_t mrep_eval_surfaces(const mrep_geom* geom, int64_t n, const int32_t* surface_id, const double* uv,
                           double* xyz_out, void* stream);

/* ---------------------------------------------------------------------- */
/* Learned seeding (an extension; the paper has no learned part)           */
/* ---------------------------------------------------------------------- */
/* A multilayer perceptron scores a query against one candidate piece of its
 * geometry (a cubic piece of a curve or a bicubic patch of a surface, the
 * Sec. 5.2 matrix representation): the local parameter(s) of the closest point
 * on the piece and the logit that the projection lies on it.  Two kinds:
 *   MREP_NN_CURVE:   x (15: the piece's 4 control points and the query)
 *                    -> 128 -> 128 -> 2 = (u, logit);          18818 parameters
 *   MREP_NN_SURFACE: x (51: the patch's 16 control points, row-major in
 *                    (i along u, j along v), and the query)
 *                    -> 128 -> 128 -> 3 = (s, t, logit);       23555 parameters
 * Inputs are translated by the control points' centroid and divided by the
 * diagonal of their axis-aligned box.  Hidden layers: Linear then GELU (erf
 * form).  Parameters: FP32, row-major W[out][in], in the order W1 b1 W2 b2 W3
 * b3.  Products run as BF16 MFMA with FP32 accumulation; master weights and
 * Adam state stay FP32.
 * Loss of a batch of B rows, outputs y[0..m-1] with m = MREP_NN_*_OUT, targets
 * t[0..m-2] and a in {0, 1}, z = y[m-1]:
 *   (1/B) sum [ a |y[0..m-2] - t|^2 + max(z, 0) - z a + log(1 + exp(-|z|)) ]. */
#define MREP_NN_CURVE 0
#define MREP_NN_SURFACE 1
#define MREP_NN_CURVE_IN 15
#define MREP_NN_CURVE_OUT 2
#define MREP_NN_SURFACE_IN 51
#define MREP_NN_SURFACE_OUT 3
#define MREP_NN_HIDDEN 128
#define MREP_NN_K 4 /* candidate pieces scored per query */

typedef struct mrep_nn mrep_nn; /* device view of a caller-owned state buffer (non-owning) */

/* Parameter count of a kind; -1 for an unknown kind. */
int32_t mrep_nn_param_count(int32_t kind);

/* Sizes for a kind: *state_bytes of the network state buffer (parameters,
 * Adam moments, gradient, packed BF16 weight image), *work_bytes of the work
 * buffer of mrep_nn_forward / mrep_nn_train_step for `batch` rows.  Either
 * output may be NULL (not both).  Errors: MREP_E_INVALID_ARG. */
int32_t mrep_nn_bytes(int32_t kind, int64_t batch, int64_t* state_bytes, int64_t* work_bytes);

/* Bind a DEVICE buffer of >= state_bytes (256-byte aligned, caller-owned,
 * must outlive the handle) as the state of a network of `kind`.  Its contents
 * are undefined until mrep_nn_init or mrep_nn_set_params.  Release the handle
 * with mrep_nn_release (the buffer stays the caller's).
 * Errors: MREP_E_INVALID_ARG, MREP_E_SMALL_BUFFER, MREP_E_NO_DEVICE. */
int32_t mrep_nn_bind(int32_t kind, void* dev_state, int64_t bytes, mrep_nn** out);
void mrep_nn_release(mrep_nn* nn);

/* Weights uniform in +-1/sqrt(fan_in) from splitmix64(seed), biases 0, Adam
 * state and step count reset.  Synchronous on `stream`. */
int32_t mrep_nn_init(mrep_nn* nn, uint64_t seed, void* stream);
/* host[n] (HOST, n = mrep_nn_param_count(kind)) -> parameters; resets Adam.
 * Synchronous on `stream`.  Errors: MREP_E_INVALID_ARG, MREP_E_HIP. */
int32_t mrep_nn_set_params(mrep_nn* nn, const float* host, int64_t n, void* stream);
/* parameters -> host[n] (HOST).  Synchronous on `stream`. */
int32_t mrep_nn_get_params(const mrep_nn* nn, float* host, int64_t n, void* stream);

/* Products of mrep_nn_forward and mrep_nn_train_step: MREP_NN_COMPUTE_BF16
 * (default; BF16 MFMA, FP32 accumulation) or MREP_NN_COMPUTE_FP32 (a debug
 * mode: plain FP32 multiply-adds, no BF16 rounding, for checking gradients
 * against an FP64 reference to ~1e-5).  mrep_nn_infer and the seeded
 * projections always run BF16.  Errors: MREP_E_INVALID_ARG. */
#define MREP_NN_COMPUTE_BF16 0
#define MREP_NN_COMPUTE_FP32 1
int32_t mrep_nn_set_compute(mrep_nn* nn, int32_t compute);

/* Outputs y[n][out] for inputs x[n][in] (both DEVICE, FP32; in, out of the
 * network's kind).  mrep_nn_forward: the training kernels (layer by layer
 * through `work`, of mrep_nn_bytes(kind, n) work bytes); mrep_nn_infer: the
 * fused inference kernel (weights in LDS, no work buffer).  Asynchronous on
 * `stream`.  Errors: MREP_E_INVALID_ARG, MREP_E_SMALL_BUFFER, MREP_E_HIP. */
int32_t mrep_nn_forward(const mrep_nn* nn, int64_t n, const float* x, float* y, void* work, int64_t work_bytes,
                        void* stream);
int32_t mrep_nn_infer(const mrep_nn* nn, int64_t n, const float* x, float* y, void* stream);

/* One training step on `batch` rows: forward, the loss above, backward, and
 * (lr > 0) one Adam step (beta = 0.9, 0.999; eps 1e-8; bias-corrected).
 * x[n_rows][in], target[n_rows][out - 1], accept[n_rows]: DEVICE FP32
 * training set.  rows[batch] (DEVICE int32, nullable) selects the rows of this
 * batch; an entry outside [0, n_rows) contributes an all-zero row.  rows ==
 * NULL: the first `batch` rows (batch <= n_rows).  loss_out (DEVICE float,
 * nullable): the batch loss before the step.  grad_out (DEVICE
 * float[param_count], nullable): the gradient.  work: DEVICE,
 * mrep_nn_bytes(kind, batch) work bytes.  Asynchronous on `stream`.
 * Errors: MREP_E_INVALID_ARG, MREP_E_SMALL_BUFFER, MREP_E_HIP. */
int32_t mrep_nn_train_step(mrep_nn* nn, int64_t n_rows, const float* x, const float* target, const float* accept,
                           int64_t batch, const int32_t* rows, float lr, float* loss_out, float* grad_out,
                           void* work, int64_t work_bytes, void* stream);

/* Workspace of mrep_project_curves_seeded and mrep_nn_features for n queries
 * (DEVICE, 256-byte aligned).  Errors: MREP_E_INVALID_ARG. */
int32_t mrep_seeded_workspace_bytes(const mrep_geom* geom, int64_t n, const mrep_opts* opts, int64_t* bytes);

/* Training-data export: for every query its MREP_NN_K candidate pieces (the
 * pieces whose bounding spheres come closest, nearest first) as curve-local
 * indices seg_out[n][4] (-1: the curve has fewer pieces, or a bad id) and
 * their MREP_NN_CURVE network inputs x_out[n][4][15].  All arrays DEVICE.  Asynchronous.
 * Errors: MREP_E_INVALID_ARG, MREP_E_SMALL_BUFFER, MREP_E_HIP. */
int32_t mrep_nn_features(const mrep_geom* geom, int64_t n, const int32_t* curve_id, const double* q_xyz,
                         int32_t* seg_out, float* x_out, void* workspace, int64_t ws_bytes, void* stream);

/* Seeded projection: same contract and outputs as mrep_project_curves (BF16
 * mode only).  The network picks one of each query's 4 candidate pieces and
 * seeds Newton there; the answer is kept only when a certificate proves it is
 * the global minimum (every other piece is farther by its bounding sphere, by
 * its endpoint distances where (C - q).C' keeps one sign on it, read off its
 * Bernstein coefficients, or by its certified piece minimum); every other query goes through the screened pipeline and is
 * flagged MREP_F_NN_FALLBACK.  nn == NULL: sphere-pruned projection, every
 * piece whose sphere lower bound reaches the best sphere upper bound is
 * refined (no fallback).  ws: mrep_seeded_workspace_bytes(n).
 * Errors: as mrep_project_curves. */
int32_t mrep_project_curves_seeded(const mrep_geom* geom, const mrep_nn* nn, const mrep_opts* opts, int64_t n,
                                   const int32_t* curve_id, const double* q_xyz, void* workspace, int64_t ws_bytes,
                                   double* t_out, double* dist_out, int32_t* seg_out, uint32_t* flags_out,
                                   void* stream);

/* Workspace of mrep_project_surfaces_seeded and mrep_nn_surface_features for
 * n queries (DEVICE, 256-byte aligned).  Errors: MREP_E_INVALID_ARG. */
int32_t mrep_surface_seeded_workspace_bytes(const mrep_geom* geom, int64_t n, const mrep_opts* opts,
                                            int64_t* bytes);

/* Training-data export for surfaces: for every query its MREP_NN_K candidate
 * patches (the smallest bounding-sphere lower bounds, nearest first) as
 * surface-local indices patch_out[n][4] (-1: the surface has fewer patches,
 * or a bad id) and their MREP_NN_SURFACE network inputs x_out[n][4][51].
 * All arrays DEVICE.  Asynchronous.
 * Errors: MREP_E_INVALID_ARG, MREP_E_SMALL_BUFFER, MREP_E_HIP. */
int32_t mrep_nn_surface_features(const mrep_geom* geom, int64_t n, const int32_t* surface_id, const double* q_xyz,
                                 int32_t* patch_out, float* x_out, void* workspace, int64_t ws_bytes, void* stream);

/* Seeded surface projection: same contract and outputs as
 * mrep_project_surfaces.  The network (kind MREP_NN_SURFACE, required) scores
 * each query's 4 candidate patches; Newton from the predicted (s, t) on the
 * best-scored patch attains a distance d_seed.  A listed patch whose sphere
 * lower bound or sampled second-order lower bound exceeds d_seed plus the tie
 * margin is dropped; the others get the certified patch minimum as in
 * mrep_project_surfaces, so the answer is the same global minimum.
 * MREP_F_NN_FALLBACK marks the queries whose minimum does not lie on the
 * seeded patch, or that took the full scan.
 * ws: mrep_surface_seeded_workspace_bytes(n).
 * Errors: as mrep_project_surfaces. */
int32_t mrep_project_surfaces_seeded(const mrep_geom* geom, const mrep_nn* nn, const mrep_opts* opts, int64_t n,
                                     const int32_t* surface_id, const double* q_xyz, void* workspace,
                                     int64_t ws_bytes, double* uv_out, double* dist_out, int32_t* patch_out,
                                     uint32_t* flags_out, void* stream);

/* ---------------------------------------------------------------------- */
/* Host introspection of the constant matrices (for tests and tools)       */
/* ---------------------------------------------------------------------- */

/* (p+1)x(p+1) row-major.  inverse = 0: B_p with [1 u .. u^p] B_p = Bernstein
 * basis row (Sec. 5.2.1, eq. bsplineafter); inverse = 1: B_p^{-1}, the
 * power-to-Bernstein matrix (Sec. 5.3, the rebasement matrix T). */
int32_t mrep_bernstein_matrix(int32_t p, int32_t inverse, double* out);

/* 2(p+1)x(p+1) row-major subdivision matrix [S_L(z); S_R(z)] of a degree-p
 * Bezier piece (Sec. 5.2.2, eqs. submatrix and subLandR, at degree p). */
int32_t mrep_subdivision_matrix(int32_t p, double z, double* out);

/* (m+1)x(n+1) row-major Gram matrix of Bernstein bases (Sec. 5.2.2, eq. gram). */
int32_t mrep_gram_matrix(int32_t m, int32_t n, double* out);

const char* mrep_last_error(void);
int32_t mrep_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MREP_H */
