/*
 * utd.h -- C ABI of the smooth-surface UTD field library (MI355X / gfx950).
 *
 * The library evaluates the receiver field of a point source in a scene of
 * triangles (occluders only) and convex PEC bodies (spheres and vertical
 * finite cylinders), with the smooth-surface diffraction of the paper
 * (Sec. II-B, Eqs. (1)-(4); Sec. III-B for which creeping paths are summed):
 *
 *   E(R) = U_LOS E^i(R) + sum_bodies [ U^r E^r(R) + sum_paths U^d E^d(R) ]
 *
 * E^i is the ray field of a Hertzian dipole, E^r the reflected field of
 * Eq. (3) with the UTD (Fock) reflection coefficients, E^d the creeping-wave
 * field of Eq. (4) with the UTD transfer coefficients; the U are the
 * Heaviside visibilities of Eqs. (1)-(2), decided against the triangle BVH
 * and against the other bodies.  Time convention e^{+j w t}; lengths in
 * metres, frequencies in Hz, c = 299792458 m/s.
 *
 * Conventions for every entry point:
 *   - Pointers documented "device" must point to GPU memory readable (and,
 *     for outputs, writable) by the current HIP device.  "host" pointers are
 *     read during the call only.  The caller owns every buffer it passes; the
 *     library never frees them.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the call returns without waiting for it.  The library's own
 *     temporary device memory is allocated and released in stream order.
 *   - A non-OK status means nothing was enqueued; utd_last_error() gives a
 *     message for the calling thread.  No exception crosses the ABI.
 *   - Conditions only visible on the device (source inside a body, receiver
 *     inside a body, receiver on a sphere's axial caustic, invalid device
 *     inputs) are reported per receiver through `rx_flags` (UTD_FLAG_*),
 *     never as a status.  Invalid device inputs also raise bits of a
 *     device-wide word read by utd_input_status; they never produce
 *     non-finite fields:
 *       receiver with a non-finite coordinate  -> E = 0 there,
 *                                                 UTD_FLAG_INVALID_RX, UTD_BAD_RX
 *       body with a non-finite parameter, radius <= 0 or height < 0
 *                                              -> E = 0 at every receiver of
 *                                                 the call (of the frame when
 *                                                 batched), UTD_FLAG_BAD_BODY,
 *                                                 UTD_BAD_BODY
 *       frequency not finite or <= 0           -> E = 0 at that frequency,
 *                                                 UTD_FLAG_BAD_FREQ on every
 *                                                 receiver, UTD_BAD_FREQ
 */
#ifndef UTD_H
#define UTD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct utd_scene utd_scene;

typedef enum {
    UTD_OK = 0,
    UTD_E_ARG = -1,          /* invalid argument (NULL, negative size, bad option) */
    UTD_E_DEVICE = -2,       /* a HIP runtime call failed */
    UTD_E_OOM = -3,          /* device or host allocation failed */
    UTD_E_UNSUPPORTED = -5   /* valid but not supported by this library */
} utd_status;

/* Per-receiver flags written to rx_flags (bit set = condition holds). */
#define UTD_FLAG_INSIDE    1u  /* receiver inside a body: E = 0                  */
#define UTD_FLAG_CAUSTIC   2u  /* a sphere creeping path dropped at the axial caustic */
#define UTD_FLAG_LOS       4u  /* direct path visible (U_LOS = 1)               */
#define UTD_FLAG_TX_INSIDE 8u  /* source inside a body: E = 0 for every receiver */
#define UTD_FLAG_INVALID_RX 16u /* receiver coordinate not finite: E = 0          */
#define UTD_FLAG_BAD_BODY  32u  /* an invalid body in the call (frame): E = 0      */
#define UTD_FLAG_BAD_FREQ  64u  /* an invalid frequency: E = 0 at that frequency   */

/* Bits of the device input-status word (utd_input_status). */
#define UTD_BAD_RX   1u
#define UTD_BAD_BODY 2u
#define UTD_BAD_FREQ 4u

typedef struct {
    int precision;          /* 0: FP32 field evaluation with FP64 path lengths and
                               phase; 1: FP64 throughout.  Default 0.          */
    int l_enc;              /* extra encirclements per side, 0..2 (Sec. III-B's
                               generalised Fermat paths).  Default 0.          */
    int bodies_occlude;     /* 1: segments are also tested against the other
                               bodies.  Default 1.                             */
    int lit_branch;         /* 1: include the direct and reflected fields
                               (Eq. (1)); 0: creeping fields only.  Default 1. */
    double caustic_guard;   /* sphere creeping paths whose receiver lies closer
                               than this to the source axis are dropped and
                               flagged (m).  Default 1e-6.                     */
    int wall_reflections;   /* 1: add one specular bounce on the scene's
                               triangle planes -- the wall's own reflected ray
                               and the body paths it feeds or that feed it
                               (utd_scene_set_wall_material); forward calls
                               only.  Default 0.                               */
    int caustic_uniform;    /* 1: a sphere's creeping paths that meet on the
                               source axis in pairs (near and far side, Sec.
                               II-B's paths around the sphere), both visible,
                               are summed by the uniform Bessel-function form
                               of their azimuthal integral instead of as two
                               rays: finite on the axis, the two rays' sum
                               away from it up to O(1/(k a eps)); paths left
                               unpaired keep caustic_guard.  Receivers with
                               theta_R > pi/2 pair at the rear axis, the
                               others at the front.  Forward calls only (the
                               adjoint entry points return
                               UTD_E_UNSUPPORTED); batched frames hold no
                               spheres.  Default 0.                            */
} utd_options;

/* Wall material of a scene's reflecting planes: a homogeneous slab of
 * relative permittivity eps_r (>= 1), conductivity sigma (S/m, >= 0) and
 * thickness (m, > 0; INFINITY for a half-space), or, with perfect_conductor
 * set, a perfect conductor (R_perp = -1, R_par = +1).  The default is 10 cm
 * of brick with ITU-R P.2040's values: eps_r 3.75, sigma 0.038 S/m. */
typedef struct {
    double eps_r;
    double sigma;
    double thickness;
    int perfect_conductor;
} utd_wall_material;

/* Bodies, device arrays of float32, row-major:
 *   sph[n_sph][4] = (cx, cy, cz, a)            sphere centre and radius
 *   cyl[n_cyl][5] = (cx, cy, z0, h, a)         vertical cylinder: axis through
 *                                              (cx, cy), lateral surface z0..z0+h,
 *                                              radius a; solid for occlusion  */
typedef struct {
    const float *sph;
    int64_t n_sph;
    const float *cyl;
    int64_t n_cyl;
} utd_bodies;

/* Point source: position (m), dipole direction (unnormalised is allowed; the
 * field scales with it) and amplitude A: E^i(P) = A (p - (p.s)s) e^{-jks}/s. */
typedef struct {
    float pos[3];
    float dipole[3];
    double amplitude;
} utd_source;

/* Fills the defaults listed above. */
void utd_default_options(utd_options *opt);

/* Builds the occluder scene: copies n_tri triangles (host float32
 * [n_tri][3][3], vertex-major) to the device and builds a BVH over them
 * (binned SAH, host C++).  Triangles lying in a face plane of the scene's
 * bounding box (a room's walls, floor and ceiling) go to a second tree that
 * only segments reaching outside the box have to walk.  n_tri may be 0.
 * *out receives the handle.
 * Errors: UTD_E_ARG (out NULL, n_tri < 0, tri NULL with n_tri > 0),
 * UTD_E_OOM, UTD_E_DEVICE. */
utd_status utd_scene_create(const float *tri_xyz, int64_t n_tri, utd_scene **out);

/* Frees the scene's device memory (waits for the device first).  NULL is a no-op. */
void utd_scene_destroy(utd_scene *scene);

/* Number of triangles and BVH nodes of a scene (for reporting). */
int64_t utd_scene_triangles(const utd_scene *scene);
int64_t utd_scene_nodes(const utd_scene *scene);

/* Reflecting planes of a scene (Eq. (3) applied to the walls, with the
 * image-source construction of a planar mirror): all triangles lying in one
 * plane n.x = d reflect as one mirror; a triangle's unit normal has its
 * first component of magnitude > 1e-9 positive, triangles whose normals and
 * offsets agree after rounding to multiples of 1e-6 share a plane, and the
 * planes are ordered by those rounded values.  Returns their number; when
 * out (host double [n][4]) is not NULL writes (n_x, n_y, n_z, d) of each. */
int64_t utd_scene_planes(const utd_scene *scene, double *out);

/* Sets the wall material of the scene's planes (see utd_wall_material).
 * Errors: UTD_E_ARG for NULL or out-of-range values. */
utd_status utd_scene_set_wall_material(utd_scene *scene, const utd_wall_material *mat);

/* Forward field (Eqs. (1)-(4)).
 *   rx       device float32 [n_rx][3]  receiver positions
 *   freqs_hz device float64 [n_f]      frequencies (> 0)
 *   E_out    device, [n_f][3][n_rx] complex, interleaved (re, im):
 *            float32 pairs when opt->precision == 0, float64 pairs when 1.
 *            Fully overwritten.
 *   rx_flags device uint8 [n_rx] or NULL.
 * n_rx == 0 or n_f == 0 enqueues nothing and returns UTD_OK.
 * Scratch (path masks and records, the candidate-path queue and visible
 * list) comes from a
 * grow-only buffer the library keeps per (device, stream) between calls,
 * allocated stream-ordered and released at process exit; calls on one stream
 * are ordered by the stream, so issuing them from several host threads at
 * once is not supported.
 * With opt->wall_reflections the receivers also get one specular bounce on
 * the scene's planes (Eq. (3) for a planar slab, image source and image
 * receiver): the wall's reflected ray (with the lit branch), and each body's
 * two primary creeping paths and its reflection fed by the wall's image
 * source (Fig. 1's equivalent source) or reaching the receiver through the
 * wall, every leg tested for visibility.
 * Errors: UTD_E_ARG for NULL pointers with non-zero sizes, n_rx < 0, n_f < 0,
 * l_enc outside 0..2, precision outside {0, 1}; UTD_E_OOM when the scratch
 * cannot be allocated; UTD_E_DEVICE on launch failure. */
utd_status utd_smooth_field(const utd_scene *scene, const utd_bodies *bodies,
                            const utd_source *tx, const float *rx, int64_t n_rx,
                            const double *freqs_hz, int n_f, const utd_options *opt,
                            void *E_out, uint8_t *rx_flags, void *stream);

/* Adjoint of utd_smooth_field (gradients for optimisation over the scene,
 * Sec. I / Sec. II-B: the field of Eqs. (1)-(4) is differentiable in the
 * body parameters and the source position wherever the visibility of every
 * path is unchanged).  For a real loss L(E) with grad_E = dL/dRe(E) + j dL/dIm(E)
 * (same layout and precision as E_out) writes
 *   d_cyl[n_cyl][3] = dL/d(cx, cy, a) per cylinder,
 *   d_sph[n_sph][4] = dL/d(cx, cy, cz, a) per sphere,
 *   d_tx[3]         = dL/d(source position),
 * i.e. dL/dtheta = Re sum conj(grad_E) dE/dtheta (PyTorch's convention for
 * complex autograd).  All three are device arrays of float32 when
 * opt->precision == 0 and float64 when 1, fully overwritten (zeros when
 * n_rx == 0 or n_f == 0).  Cylinder heights (z0, h) only move visibility
 * boundaries and get no gradient.  Path classification and visibility are
 * those of the forward evaluation at the same inputs and are held fixed;
 * receivers inside a body or with the source inside one contribute nothing.
 * The reduction over receivers and frequencies runs in FP64 in a fixed order
 * (bitwise reproducible).  Uses the per-stream scratch of
 * utd_smooth_field.
 * Errors as for utd_smooth_field; UTD_E_ARG if d_tx is NULL, d_cyl / d_sph is
 * NULL with a non-zero count, or grad_E is NULL with n_rx, n_f > 0;
 * UTD_E_UNSUPPORTED with opt->wall_reflections. */
utd_status utd_smooth_field_backward(const utd_scene *scene, const utd_bodies *bodies,
                                     const utd_source *tx, const float *rx, int64_t n_rx,
                                     const double *freqs_hz, int n_f, const utd_options *opt,
                                     const void *grad_E, void *d_cyl, void *d_sph, void *d_tx,
                                     void *stream);

/* Forward evaluation that keeps its classification for the adjoint.  Same
 * inputs, outputs and errors as utd_smooth_field (rx_flags may be NULL), and
 * additionally *state receives a handle owning one device allocation (made
 * stream-ordered on `stream`) with the call's body and frequency constants,
 * path masks, path records, flags and the adjoint's scratch, and copies of
 * rx and the bodies; the caller's arrays may change afterwards.
 * utd_smooth_field_backward_saved(state, ...) then gives exactly the
 * gradients of utd_smooth_field_backward at the forward's inputs (the same
 * kernels on the same masks and records, bitwise equal) without repeating
 * the classification and visibility pass.  The state is read-only for the
 * backward, which may be called several times; a backward on another stream
 * must be ordered after the forward by the caller.  Release with
 * utd_forward_state_release (NULL-safe): the buffer is kept for reuse by the
 * next saved forward on `stream` (one per device and stream, the largest
 * seen; a smaller one is freed stream-ordered on `stream`), so steady-state
 * training steps allocate nothing; the kept buffer lives until the process
 * ends.  Memory held per
 * state: the forward's workspace, about (80 B FP32 / 120 B FP64)
 * x (2 l_enc + 3) x n_rx x n_bodies for the records plus 64 B per possible
 * path for the adjoint.
 * Errors: those of utd_smooth_field; UTD_E_ARG for a NULL state pointer;
 * UTD_E_UNSUPPORTED with opt->wall_reflections; UTD_E_OOM when the state
 * cannot be allocated (*state is NULL after any error). */
typedef struct utd_forward_state utd_forward_state;
utd_status utd_smooth_field_saved(const utd_scene *scene, const utd_bodies *bodies,
                                  const utd_source *tx, const float *rx, int64_t n_rx,
                                  const double *freqs_hz, int n_f, const utd_options *opt,
                                  void *E_out, uint8_t *rx_flags, utd_forward_state **state,
                                  void *stream);
/* Errors: UTD_E_ARG for a NULL state or d_tx, d_cyl / d_sph NULL with a
 * non-zero count, grad_E NULL with work; UTD_E_DEVICE on launch failure. */
utd_status utd_smooth_field_backward_saved(const utd_forward_state *state, const void *grad_E,
                                           void *d_cyl, void *d_sph, void *d_tx, void *stream);
utd_status utd_forward_state_release(utd_forward_state *state, void *stream);

/* Many frames in one launch (dynamic scenes: a moving crowd over a static
 * room, Sec. III; the field of every frame is that of utd_smooth_field with
 * the frame's cylinders as bodies).  Frame f has the cylinders
 * cyl[body_off[f] .. body_off[f+1]) and the receivers rx[rx_off[f] .. rx_off[f+1]);
 * all frames share the scene triangles, the source and the frequencies.
 *   body_off, rx_off  device int64 [n_frames + 1], non-decreasing, starting at 0
 *   cyl               device float32 [n_cyl][5] (cx, cy, z0, h, a)
 *   rx                device float32 [n_rx][3]
 *   E_out             device complex, precision as utd_smooth_field; frame f
 *                     occupies the [n_f][3][n_rx_f] block that starts at complex
 *                     element 3 * n_f * rx_off[f] (frames concatenated)
 *   rx_flags          device uint8 [n_rx] or NULL
 * Offsets are clamped to [0, n_cyl] / [0, n_rx] and to non-decreasing values
 * on the device, so malformed offsets give empty frames, never out-of-bounds
 * accesses.  One work queue over (frame, tile of receivers) feeds a
 * persistent kernel; the call replays a captured HIP graph (the constants,
 * receiver order, body grids, source-side profiles, receiver flags and the
 * persistent kernel: six launches) as long as its arguments repeat (device
 * data may change), and when the stream is itself being captured it records
 * the six launches into the caller's graph instead (the workspace must then exist from an earlier call
 * of at least this size).  A caller's graph points into that workspace: once
 * a call has been captured, a later call that needs a larger workspace
 * allocates a new one and keeps the old one alive until the process ends, so
 * captured graphs stay valid.  Tile shape: utd_batched_config.  The library keeps
 * one workspace per device: concurrent batched calls on one device race.
 * Errors as for utd_smooth_field; UTD_E_ARG for n_frames < 0, n_cyl < 0, NULL
 * offsets with n_frames, n_rx, n_f > 0, or a capture without workspace;
 * UTD_E_UNSUPPORTED with opt->wall_reflections. */
utd_status utd_smooth_field_batched(const utd_scene *scene, int64_t n_frames,
                                    const int64_t *body_off, const float *cyl, int64_t n_cyl,
                                    const int64_t *rx_off, const float *rx, int64_t n_rx,
                                    const utd_source *tx, const double *freqs_hz, int n_f,
                                    const utd_options *opt, void *E_out, uint8_t *rx_flags,
                                    void *stream);

/* Tile shape of utd_smooth_field_batched: receivers per work item (64, 128
 * or 256; one lane per receiver) and resident workgroups per compute unit of
 * the persistent grid (1..16; default 256 and 3).  Chosen by the autotuner
 * of the Python package; applies to later calls.  Errors: UTD_E_ARG for
 * other values. */
utd_status utd_batched_config(int tile_rx, int blocks_per_cu);

/* Allocation-free variant of utd_smooth_field, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * utd_smooth_field; it calls no allocating routine.  Its scratch (path
 * masks and records, the candidate queue, body and frequency constants) is
 * one static device array of 256 MiB per device, which every call on that
 * device shares and which the device keeps until the process ends: calls
 * that overlap on one device (several streams or host threads at once)
 * race.  A call whose scratch would exceed 256 MiB returns UTD_E_ARG and
 * enqueues nothing (with l_enc = 0 the FP32 path takes about 460 bytes per
 * (receiver, body) pair plus 72 per receiver: 65 536 receivers with one
 * sphere fit, and so do 16 384 receivers with 32 bodies). */
utd_status utd_smooth_field_noalloc(const utd_scene *scene, const utd_bodies *bodies,
                                    const utd_source *tx, const float *rx, int64_t n_rx,
                                    const double *freqs_hz, int n_f, const utd_options *opt,
                                    void *E_out, uint8_t *rx_flags, void *stream);

/* Path census (reporting): runs the classification and visibility stage of
 * utd_smooth_field for the same inputs and writes, to the host array
 * counts[10], the number of (receiver, body) pairs with each mask bit set --
 * counts[2*ell + s] creeping paths on side s (0: towards the receiver,
 * 1: far side) with ell encirclements, counts[6] reflections, counts[7]
 * caustic drops -- then counts[8] receivers with a visible direct path and
 * counts[9] receivers inside a body.  Waits for the stream.  With
 * opt->caustic_uniform the census is taken before the pairing: both paths
 * of a pair count, and no path is dropped at the caustic (the guard applies
 * after pairing, to paths left alone).
 * Errors as for utd_smooth_field; UTD_E_ARG if counts is NULL. */
utd_status utd_path_census(const utd_scene *scene, const utd_bodies *bodies, const utd_source *tx,
                           const float *rx, int64_t n_rx, const utd_options *opt, int64_t *counts,
                           void *stream);

/* Per-(receiver, body) path masks of the visibility stage: runs the
 * classification and visibility of utd_smooth_field for the same inputs and
 * options (the decisions depend on opt->precision) and writes
 *   mask_out  device uint8 [n_bodies][n_rx], body-major (spheres first, then
 *             cylinders, as in `bodies`): bit 2*ell + s set when the creeping
 *             path of side s (0: towards the receiver, 1: far side) with ell
 *             encirclements exists and both its legs are visible (the U^d of
 *             Eq. (2)); bit 6 the same for the reflection (U^r of Eq. (1));
 *             bit 7 when a sphere creeping path was dropped at the axial
 *             caustic;
 *   rx_flags  device uint8 [n_rx] or NULL (UTD_FLAG_*, UTD_FLAG_LOS = U_LOS).
 * These are the decisions utd_smooth_field takes for the same inputs; tests
 * feed them to an independent evaluation to compare fields path by path.
 * With opt->caustic_uniform the masks are those before the pairing (as for
 * utd_path_census).
 * Asynchronous on `stream`.  Errors as for utd_smooth_field; UTD_E_ARG if
 * mask_out is NULL with bodies and receivers. */
utd_status utd_path_masks(const utd_scene *scene, const utd_bodies *bodies, const utd_source *tx,
                          const float *rx, int64_t n_rx, const utd_options *opt, uint8_t *mask_out,
                          uint8_t *rx_flags, void *stream);

/* Wall-bounce decisions of utd_smooth_field with wall reflections for the
 * same inputs: for every (receiver, plane) a 64-bit word, device uint64
 * [n_rx][n_planes] (planes as utd_scene_planes orders them): bit 0 the
 * wall's own reflected ray visible; for body b (spheres first, then
 * cylinders) bits 1 + 6 b + k: k = 0, 1 the creeping path of side + / - fed
 * by the wall, 2 the body reflection fed by the wall, 3, 4 the creeping path
 * of side + / - reaching the receiver through the wall, 5 the body
 * reflection reaching it through the wall.  Asynchronous on `stream`.
 * Errors as for utd_smooth_field; UTD_E_UNSUPPORTED for more than 10 bodies;
 * UTD_E_ARG if mask_out is NULL with planes and receivers. */
utd_status utd_wall_masks(const utd_scene *scene, const utd_bodies *bodies, const utd_source *tx,
                          const float *rx, int64_t n_rx, const utd_options *opt, uint64_t *mask_out,
                          void *stream);

/* Device input status: waits for the current device, writes to *bits the OR
 * of the UTD_BAD_* bits raised by every call on this device since the last
 * read (invalid receivers, bodies or frequencies found by the kernels), and
 * clears them.  The calls themselves never wait for this.  Errors: UTD_E_ARG
 * for NULL, UTD_E_DEVICE. */
utd_status utd_input_status(uint32_t *bits);

/* Per-kernel timing for measurement.  utd_profile_enable(1) makes every
 * later call record a HIP event pair around each kernel it launches, on the
 * stream it launches on; utd_profile_read waits for those events, writes the
 * summed durations in milliseconds and launch counts into ms[k] and count[k]
 * (k = UTD_K_*; arrays of UTD_K_COUNT entries, host) and clears the record.
 * utd_profile_enable(0) stops recording.  While recording, a batched call
 * launches its kernels directly instead of replaying its graph, and times
 * its constants, receiver order, body grids, source-side profiles and the
 * receivers' flags and direct rays (UTD_K_PREP) apart from its persistent
 * kernel (UTD_K_BATCHED).  Not for concurrent use from several host
 * threads.  Errors: UTD_E_ARG for NULL outputs, UTD_E_DEVICE. */
#define UTD_K_PREP 0
#define UTD_K_OCCLUDE 1
#define UTD_K_FIELD 2
#define UTD_K_BACKWARD 3
#define UTD_K_REDUCE 4
#define UTD_K_BATCHED 5
#define UTD_K_WALLS 6
#define UTD_K_CAUSTIC 7
#define UTD_K_COUNT 8
void utd_profile_enable(int on);
utd_status utd_profile_read(double *ms, int64_t *count);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char *utd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* UTD_H */
