/*
 * props.h — C ABI of the MI355X real-fluid property library (libprops.so).
 *
 * Per-cell thermophysical properties of a supercritical multi-species mixture, as a
 * pressure-based reacting-flow solver requests them once per pressure-correction loop
 * (Section 2 of "Detailed simulation of LOX/GCH4 flame-vortex interaction in
 * supercritical Taylor-Green flows with machine learning"), and the neural-network
 * surrogate that replaces them (Section 4).
 *
 * Conventions for every call:
 *   - SI units.  h and e are mass-specific and absolute (they include the enthalpy of
 *     formation), cp in J/(kg K), sound speed c in m/s, mu in Pa s, lambda in W/(m K).
 *   - Arrays are structure-of-arrays device pointers (hipMalloc'd or any device tensor),
 *     unless the argument says "host".  Y is species-major: Y[i * n + k] is the mass
 *     fraction of species i in cell k.  The caller owns every array; the library owns only
 *     its handles and the device copies of tables and weights it builds.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  Property calls are
 *     asynchronous on that stream and never synchronise the host.
 *   - Return codes: 0 = OK, negative = PROPS_E*; props_last_error() then describes the
 *     failure (thread-local, valid until the next failing call on the same thread).
 *   - Per-cell outcome flags go to an optional uint8 status array (PROPS_ST_*).
 */
#ifndef PROPS_H
#define PROPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ error codes */
enum {
    PROPS_OK = 0,
    PROPS_EINVAL = -1,    /* bad argument (null handle, n < 0, unsupported mode ...) */
    PROPS_ENOMEM = -2,    /* device or host allocation failed */
    PROPS_EHIP = -3,      /* a HIP runtime call failed (message names it) */
    PROPS_ETOOBIG = -4,   /* request exceeds a fixed limit (species count, budget, cell
                           * count: props_pr, props_diffusion and props_features_hpz take
                           * n <= 2^32 - 256 = 4294967040, one lane per cell, because one
                           * dispatch holds at most 2^32 - 1 work-items; props_dnn and
                           * props_dnn_features n <= 2^31 - 1, a 32-bit cell index) */
    PROPS_ETIMEDOUT = -5, /* serve_wait ran out of time */
    PROPS_ENOTREADY = -6  /* object not in a usable state (e.g. network not trained) */
};

/* ------------------------------------------------------------------ per-cell status bits */
enum {
    PROPS_ST_NONPHYS = 1,      /* NaN input, Y_i < -1e-12, |sum Y - 1| > 1e-6, rho/T/P <= 0,
                                  v <= b_m, or no root above B; outputs are NaN */
    PROPS_ST_NEWTON_MAXIT = 2, /* T inversion hit the iteration limit; outputs at last iterate */
    PROPS_ST_BRACKET = 4,      /* the temperature solving e(T) = e* is outside [60, 5000] K;
                                  outputs are NaN */
    PROPS_ST_THREE_ROOT = 8,   /* (P,T,Y): the cubic had three roots above B */
    PROPS_ST_GIBBS_TIE = 16,   /* liquid- and vapour-like roots tie in Gibbs energy to 1e-12;
                                  the larger Z was taken */
    PROPS_ST_CV_NONPOS = 32,   /* c_v <= 0 at the solution (mechanically odd state) */
    PROPS_ST_OUT_OF_HULL = 64, /* surrogate: input outside the training box */
    PROPS_ST_FALLBACK = 128    /* surrogate: cell recomputed by the PR path */
};

/* ------------------------------------------------------------------ mechanism */
/* Raw constants of one species (host struct).  W kg/mol, Tc K, Pc Pa, Vc m^3/mol,
 * omega acentric factor, dipole debye, kappa Chung association factor, Tmid K (NASA-7
 * range switch; every species of a mechanism must share one), nasa_lo/nasa_hi the seven
 * NASA coefficients below/above Tmid (a7 is not used). */
typedef struct {
    double W, Tc, Pc, Vc, omega, dipole, kappa, Tmid;
    double nasa_lo[7], nasa_hi[7];
} props_species_desc;

typedef struct props_mech_s *props_mech_t;

#define PROPS_MAX_SPECIES 8

/* Build the device tables of a mechanism: Peng-Robinson a_c, b, kappa(omega) of
 * Section 2 / Eq. (1) with the exact critical-point Omega constants, the van der Waals
 * mixing matrix 1 - k_ij, NASA-7 coefficients, and Chung's per-species and pair constants.
 * sp: host array of ns descriptors (copied).  kij: host ns*ns row-major binary-interaction
 * matrix (symmetric, zero diagonal) or NULL for all zero.  ns in 1..PROPS_MAX_SPECIES.
 * On success *out holds a handle bound to the current device. */
int props_mech_create(const props_species_desc *sp, int ns, const double *kij,
                      props_mech_t *out);
void props_mech_destroy(props_mech_t m);
int props_mech_num_species(props_mech_t m);

/* Iteration options of the (rho, e, Y) and (h, P, Y) inversions: max_iter >= 1 (default
 * 100) and the relative step size that ends the iteration (default 1e-10): a Newton-type
 * step at most this small is the last one (convergence is cubic for (rho, e, Y), which
 * takes Chebyshev's third-order step, and quadratic for (h, P, Y)); after a bisection step
 * that small, one more step is taken.  (h, P, Y) also ends after three Newton steps of
 * consistent quadratic contraction once the error they predict is below 1e-5 rtol T, and
 * (rho, e, Y) after two Chebyshev steps d1, d once the error cubic convergence predicts,
 * d^4/d1^3, is below 1e-8 rtol T.
 * max_iter and rtol outside [1, 10000] and (0, 1) return PROPS_EINVAL. */
int props_mech_set_newton(props_mech_t m, int max_iter, double rtol);

/* ------------------------------------------------------------------ property evaluation */
enum { PROPS_PTY = 0, PROPS_RHOEY = 1, PROPS_HPY = 2 };
enum { PROPS_FP64 = 0, PROPS_MIXED = 1 };

/* Device input arrays, n cells each (Y: ns*n). Unused members may be NULL. */
typedef struct {
    const double *P;       /* Pa       (PROPS_PTY, PROPS_HPY) */
    const double *T;       /* K        (PROPS_PTY) */
    const double *rho;     /* kg/m^3   (PROPS_RHOEY) */
    const double *e;       /* J/kg     (PROPS_RHOEY) */
    const double *Y;       /* [ns][n]  (every mode) */
    const double *T_guess; /* K, optional start of the T inversion (PROPS_RHOEY, PROPS_HPY) */
    const double *h;       /* J/kg     (PROPS_HPY) */
} props_in;

/* Device output arrays, n cells each.  A NULL member is not computed or written; with
 * mu, lambda and alpha all NULL the transport model is skipped entirely.  iters (optional,
 * PROPS_RHOEY and PROPS_HPY) receives the number of residual evaluations the inversion
 * took, saturated at 255.  The solver outputs of Section 4.1:
 *   psi   = (d rho / d P) at constant h and Y, s^2/m^2;
 *   alpha = lambda / (rho cp), the thermal diffusivity, m^2/s;
 *   hRT   = h_i/(R T) of each species' ideal-gas standard state (NASA polynomial),
 *           [ns][n] species-major like Y. */
typedef struct {
    double *T, *P, *Z, *rho, *h, *e, *cp, *c, *mu, *lambda;
    uint8_t *iters;
    double *psi, *alpha, *hRT;
} props_out;

/* Evaluate the Peng-Robinson property path on n independent cells.
 *   PROPS_PTY:   given P, T, Y: solve the cubic of Eq. (1) for Z, choose among physical
 *                roots (Z > B) by minimum Gibbs energy, then rho, h, e, cp, c (+ mu, lambda).
 *   PROPS_RHOEY: given rho, e, Y: find T with e(T; v = W/rho, Y) = e* by a bracketed
 *                Newton-type (Chebyshev) iteration on [60, 5000] K, then P from Eq. (1) and
 *                every property.
 *   PROPS_HPY:   given h, P, Y (the state of the pressure-based solver, Section 3): find T
 *                with h(T; P, Y) = h* by bracketed Newton iteration on [60, 5000] K, the
 *                cubic and root choice of PROPS_PTY inside every evaluation, the slope
 *                being the real-fluid cp; then every property at (P, T).  Where the chosen
 *                root switches (a subcritical two-phase gap) h(T) jumps; an h* inside the
 *                jump has no root and the iteration ends at the switch temperature.
 *   PROPS_FP64:  every step in double precision.
 *   PROPS_MIXED: mixing sums, departure functions and transport in single precision;
 *                the cubic (discriminant and root polish), the ideal-gas energy and the
 *                Newton residual stay in double.  Inputs and outputs are double either way.
 * status: optional device uint8[n] (PROPS_ST_* bits).  Asynchronous on hip_stream. */
int props_pr(props_mech_t m, int mode, int prec, const props_in *in, const props_out *out,
             int64_t n, uint8_t *status, void *hip_stream);

/* Mixture-averaged diffusion coefficients D_i [m^2/s] of every species (Section 2, the
 * species transport closure), low-pressure Chapman-Enskog form:
 *   D_ij = (3/16) sqrt(2 pi (k T)^3 / m_ij) / (P pi sigma_ij^2 Omega_D(k T / eps_ij)),
 *   D_i  = (1 - Y_i) / sum_{j != i} X_j / D_ij,   D_i = 0 if no other species is present,
 * with m_ij the reduced molecular mass, Neufeld's fit of the collision integral Omega_D,
 * Lennard-Jones parameters from Chung's critical-point relations (sigma_i = 0.809
 * Vc_i^(1/3), eps_i/k = Tc_i/1.2593) combined by Lorentz-Berthelot.  Takahashi's
 * high-pressure correction is not applied.
 * P [n] (Pa), T [n] (K), Y [ns][n] species-major, D [ns][n] species-major: device
 * arrays owned by the caller.  prec = PROPS_FP64, or PROPS_MIXED for the pair sums in
 * single precision.  Cells with NaN or non-positive P or T, Y_i < -1e-12 or
 * |sum Y - 1| > 1e-6 get D = NaN and PROPS_ST_NONPHYS in the optional status [n];
 * other cells get status 0.  Asynchronous on hip_stream.  Returns PROPS_EINVAL for a
 * NULL mechanism or array, an unknown precision or n < 0. */
int props_diffusion(props_mech_t m, int prec, const double *P, const double *T, const double *Y,
                    double *D, int64_t n, uint8_t *status, void *hip_stream);


/* ------------------------------------------------------------------ MLP surrogate */
/* The surrogate of Section 4: a multilayer perceptron with GELU activations.  The default
 * network maps a cell's (P, T, Y_1..Y_8) to (rho, h, cp, c, mu, lambda), 10 -> 4 x 256 -> 6;
 * networks of the paper's shape (3 hidden layers, Section 4.1) and with fewer outputs are
 * made with props_dnn_create_ex.  Inputs are min-max scaled to [0, 1] by the training box;
 * outputs are predicted as min-max scaled targets, with the outputs flagged in the network's
 * log mask (by default rho, cp, mu, lambda) log-transformed first (the Box-Cox transform with
 * lambda = 0 that Section 4.2 applies to density).  Matrix products run on the BF16 matrix
 * cores with FP32 accumulation; FP32 master weights; the bias is added exactly. */
typedef struct props_dnn_s *props_dnn_t;

#define PROPS_DNN_IN 10
#define PROPS_DNN_OUT 6         /* largest output count */
#define PROPS_DNN_HIDDEN 256
#define PROPS_DNN_LAYERS 5      /* weight layers of the default network: 10->256, 3 x 256->256, 256->6 */

/* Create a network on the current device with weights and biases drawn
 * U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a splitmix64 stream seeded by `seed`, and
 * identity scalers (inputs and targets taken as already in [0, 1]).  props_dnn_create makes
 * the default 4-hidden-layer, 6-output network; props_dnn_create_ex takes hidden_layers in
 * {3, 4} and outputs in 1..PROPS_DNN_OUT (other values: PROPS_EINVAL). */
int props_dnn_create(uint64_t seed, props_dnn_t *out);
int props_dnn_create_ex(uint64_t seed, int hidden_layers, int outputs, props_dnn_t *out);
void props_dnn_destroy(props_dnn_t net);
int props_dnn_get_shape(props_dnn_t net, int *hidden_layers, int *outputs);

/* Host copies of weight layer l (0..hidden_layers): W row-major [out][in] FP32 (out x in =
 * 256x10, then 256x256 for each further hidden layer, then outputs x 256) and b[out].
 * set_layer resets the Adam moments of the layer. */
int props_dnn_get_layer(props_dnn_t net, int l, float *W, float *b);
int props_dnn_set_layer(props_dnn_t net, int l, const float *W, const float *b);

/* Host scalers: in_lo/in_hi[10] raw input box (also the hull: a cell is inside when every
 * feature lies in [lo, hi] to 1e-9 of the range, or, for a feature with lo = hi, within
 * 1e-9 max(1, |lo|) of lo; such a feature scales to 0), out_lo/out_hi[6] box of
 * the transformed targets. */
int props_dnn_get_scalers(props_dnn_t net, double *in_lo, double *in_hi, double *out_lo, double *out_hi);
int props_dnn_set_scalers(props_dnn_t net, const double *in_lo, const double *in_hi,
                          const double *out_lo, const double *out_hi);

/* Which of the six outputs the network is trained on, and predicts, as a logarithm: bit j
 * for output j.  The default 0x35 (outputs 0, 2, 4, 5) is that of the (P, T, Y) surrogate
 * (rho, cp, mu, lambda log-transformed; h and c linear) and the only mask props_dnn
 * accepts; networks trained on other targets (for instance diffusion coefficients, all
 * positive and spanning decades) set their own mask before train_dnn, which fits the
 * output box on the transformed targets, and are evaluated with props_dnn_features.
 * Returns PROPS_EINVAL for bits beyond output 5.  Changing the mask of a trained network
 * invalidates its output box. */
int props_dnn_set_log_outputs(props_dnn_t net, unsigned mask);
int props_dnn_get_log_outputs(props_dnn_t net, unsigned *mask);

/* Checkpoint: network shape, FP32 master weights, Adam moments and step, epoch counter,
 * log-output mask, scalers.
 * A load followed by further training continues bit for bit. */
int props_dnn_save(props_dnn_t net, const char *path);
int props_dnn_load(const char *path, props_dnn_t *out);

/* Evaluate the surrogate on n cells given (P, T, Y) (in->P, in->T, in->Y; other members
 * ignored); writes out->rho, h, cp, c, mu, lambda (NULL members skipped; T, P, Z, e are
 * not produced).  Cells outside the training box or with non-physical inputs get
 * PROPS_ST_OUT_OF_HULL; if `fallback` is not NULL they are recomputed by
 * props_pr(PROPS_PTY, PROPS_MIXED) on the device and also get PROPS_ST_FALLBACK, without a
 * host synchronisation.  The network must share the mechanism's species order.
 * Asynchronous on hip_stream.  With a fallback the call
 * keeps its list of flagged cells in a buffer of the handle, grown (hipMalloc, after
 * synchronising hip_stream) when n exceeds every previous call: calls on one handle must
 * therefore not overlap on different streams (serialise them, or use one handle per
 * stream; the server keeps a list per slot). */
int props_dnn(props_dnn_t net, props_mech_t fallback, const props_in *in, const props_out *out,
              int64_t n, uint8_t *status, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): props_dnn with the same arguments,
 * outputs and status, whose fallback list (a count and up to n cell indices) lives in a
 * static device array of the library instead of a buffer of the handle.  It calls no
 * hipMalloc, hipFree or allocating library routine.  n <= PROPS_DNN_NOALLOC_MAX_CELLS
 * (larger: PROPS_ETOOBIG, nothing launched).  The array takes 16 MiB + 256 B on each
 * device the library runs on, held until the process ends; every call on a device shares
 * it and it keeps the last call's contents (the call resets the count on hip_stream before
 * use), so calls that overlap on one device, from any stream or thread, race.  Call with
 * the device of the network and mechanism current; otherwise PROPS_EINVAL. */
#define PROPS_DNN_NOALLOC_MAX_CELLS 4194304
int props_dnn_noalloc(props_dnn_t net, props_mech_t fallback, const props_in *in, const props_out *out,
                      int64_t n, uint8_t *status, void *hip_stream);

/* Evaluate the surrogate on raw features: X is a device array [PROPS_DNN_IN][n] (feature-
 * major, double), Y a device array [outputs][n] that receives the network's outputs in the
 * network's target units (outputs trained on their logarithm, see
 * props_dnn_set_log_outputs, are returned through exp).  Inputs are min-max scaled by the network's input box; no hull
 * test, status or fallback.  This is the entry for networks trained on other inputs than
 * (P, T, Y), such as the (h, P, Z) features below.  Asynchronous on hip_stream. */
int props_dnn_features(props_dnn_t net, const double *X, double *Y, int64_t n, void *hip_stream);

/* The inputs of the paper's surrogate (Section 4.1): enthalpy, pressure and Bilger's
 * mixture fraction of the previous iterate, the latter Box-Cox transformed (Section 4.2).
 * Bilger's coupling function beta = 2 Y_C/W_C + Y_H/(2 W_H) - Y_O/W_O is, per species i with
 * c_i, h_i, o_i carbon, hydrogen and oxygen atoms and molar mass W_i, beta = sum_i Y_i b_i with
 * b_i = (2 c_i + h_i / 2 - o_i) / W_i; Z = (beta - b_ox) / (b_fuel - b_ox) for the pure
 * species `fuel` and `oxidizer`, clamped below at 0; BC(Z) = (Z^lambda - 1) / lambda with
 * 0 < lambda <= 1 (a power transform spreading the many small values; lambda = 0, the
 * logarithm, is refused because Z = 0 occurs in pure oxidizer).
 *   atoms: host [ns][3] (C, H, O per molecule); W: host [ns] kg/mol;
 *   h, P: device [n]; Y: device [ns][n];
 *   X: device [PROPS_DNN_IN][n] <- X[0] = h, X[1] = P, X[2] = BC(Z), X[3..] = 0.
 * Asynchronous on hip_stream. */
int props_features_hpz(const int *atoms, const double *W, int ns, int fuel, int oxidizer, double bc_lambda,
                       const double *h, const double *P, const double *Y, int64_t n, double *X,
                       void *hip_stream);

/* ------------------------------------------------------------------ training */
typedef struct {
    int epochs;          /* epochs to run in this call */
    int total_epochs;    /* horizon of the cosine learning-rate schedule (0 = epochs) */
    int batch;           /* samples per step (multiple of 256; default 65536 if 0) */
    float lr, lr_min;    /* Adam learning rate, cosine-decayed from lr to lr_min */
    float beta1, beta2, eps;
    uint64_t seed;       /* per-epoch sample permutations derive from (seed, epoch) */
    int fit_scalers;     /* 1: set the input box and target box from this data first */
} props_train_cfg;

typedef struct {
    int epochs_run;
    int64_t steps;       /* optimizer steps taken in this call */
    double seconds;      /* wall time of the call */
    double samples_per_s;
    float *loss;         /* host array of >= epochs floats (may be NULL): mean L1 loss of
                            each epoch on the scaled targets */
} props_train_report;

/* Train with the L1 loss of Section 4.3 (the mean absolute error over the network's outputs)
 * and Adam.  X: device float [10][n] raw inputs (P, T, Y_1..8 for the default network),
 * feature-major; Y: device float [outputs][n] raw targets (rho, h, cp, c, mu, lambda for the
 * default network).  The call allocates a device copy of the set as 64-byte sample rows (n x 64
 * bytes, freed before it returns), from which the per-epoch permutation reads.
 * Blocking: returns when training is done (synchronises hip_stream once per epoch). */
int train_dnn(props_dnn_t net, const float *X, const float *Y, int64_t n,
              const props_train_cfg *cfg, props_train_report *rep, void *hip_stream);

/* One forward/backward pass without an update: the mean L1 loss of samples [0, n) and the
 * gradient of every weight and bias, written to the host array grad in layer order
 * (W_0, b_0, ..., W_L, b_L; shapes as in props_dnn_get_layer).  n <= 65536. */
int props_dnn_grad(props_dnn_t net, const float *X, const float *Y, int64_t n, float *grad,
                   float *loss, void *hip_stream);


/* ------------------------------------------------------------------ serving */
/* A request loop for concurrent solver subdomains (paper, Section 4.4: property inference
 * served by a GPU beside the solver).  Requests carry device arrays (PROPS_MEM_DEVICE, the
 * default), evaluated in place, or host arrays (PROPS_MEM_HOST; pinned memory, e.g.
 * hipHostMalloc, makes the copies asynchronous) staged through device slots.  The server
 * owns a device arena of `mem_budget` bytes cut into slots of `chunk_cells` cells; each
 * request is split into chunks that are admitted as slots free up, round-robin across the
 * active requests (a small request never waits for a large one to finish), and evaluated
 * (host requests: copied in, evaluated, copied out) on a pool of streams so chunks of
 * different requests overlap on the device.  A slot holds a chunk's staging buffers and its
 * fallback list, so the number of slots bounds the chunks in flight.  Mechanism tables and
 * network weights stay resident.  A cell's result does not depend on which chunk, slot or
 * stream carried it. */
typedef struct props_server_s *props_server_t;

enum { PROPS_ROUTE_PR_FP64 = 0, PROPS_ROUTE_PR_MIXED = 1, PROPS_ROUTE_DNN = 2 };
enum { PROPS_MEM_DEVICE = 0, PROPS_MEM_HOST = 1 };
enum { PROPS_EXEC_GPU = 0, PROPS_EXEC_MOCK = 1 };

typedef struct {
    int64_t mem_budget;       /* device bytes for chunk slots (>= one slot) */
    int64_t chunk_cells;      /* cells per slot (default 262144 if 0) */
    int max_inflight;         /* chunk cap in flight (0 = as many as slots) */
    int streams;              /* HIP streams in the pool (default 4 if 0) */
    int executor;             /* PROPS_EXEC_GPU, or PROPS_EXEC_MOCK: host threads stand in
                                 for the device (scheduler tests without a GPU) */
    double mock_ns_per_cell;  /* mock executor: simulated evaluation time per cell */
    int mock_species;         /* mock executor without a mechanism: species count (default 8) */
} props_serve_cfg;

typedef struct {
    int mode;                 /* PROPS_PTY, PROPS_RHOEY or PROPS_HPY (PROPS_ROUTE_DNN: PTY only) */
    int route;                /* PROPS_ROUTE_* */
    int64_t n;
    props_in in;              /* Y: [ns][n] */
    props_out out;            /* NULL members are not returned.  PROPS_ROUTE_DNN returns rho,
                                 h, cp, c, mu and lambda only (any other member: EINVAL);
                                 psi, alpha, hRT and iters need PROPS_MEM_DEVICE */
    uint8_t *status;          /* optional */
    int memory;               /* PROPS_MEM_DEVICE: in, out and status are device arrays on
                                 the server's device; PROPS_MEM_HOST: host arrays */
} props_request;

typedef struct {
    int rc;                   /* 0 or a negative PROPS_E* code */
    int64_t n;
    double t_submit, t_done;  /* seconds since the server started */
    double latency_s;
} props_result;

typedef struct {
    int64_t submitted, completed, failed, queued_requests, inflight_chunks;
    int64_t cells_done, slots, slot_bytes;
    double elapsed_s, cells_per_s;   /* since the first submission */
    double p50_s, p99_s, mean_s, max_s;   /* request latency, completed requests */
} props_serve_stats;

/* mech is required (except by the mock executor); dnn may be NULL (then PROPS_ROUTE_DNN
 * is refused).  The server does not own mech or dnn, which must outlive it.  The mock
 * executor evaluates a fixed function of each cell's inputs on host threads (it takes
 * PROPS_MEM_HOST requests only), and fails a chunk whose first input value is NaN (to
 * exercise failure paths). */
int serve_create(const props_serve_cfg *cfg, props_mech_t mech, props_dnn_t dnn,
                 props_server_t *out);
/* Thread-safe and non-blocking.  The request's arrays must stay valid (and, for device
 * requests, unmodified by the caller) until serve_wait reports it done; a device request's
 * input arrays must be ready when it is submitted (the server's streams do not wait on the
 * caller's). */
int serve_submit(props_server_t s, const props_request *req, uint64_t *ticket);
/* Wait for a ticket (timeout_us < 0: forever).  PROPS_ETIMEDOUT if not done in time;
 * otherwise the ticket is retired and res (if not NULL) filled. */
int serve_wait(props_server_t s, uint64_t ticket, int64_t timeout_us, props_result *res);
int serve_stats(props_server_t s, props_serve_stats *st);
/* Drains everything in flight, then frees the server. */
void serve_destroy(props_server_t s);

/* ------------------------------------------------------------------ measurement */
/* Not part of the method: a streaming device-to-device copy of `bytes` bytes (src and dst
 * device pointers, 16-byte aligned, not overlapping), the measured bandwidth ceiling that the
 * property kernels' HBM traffic is reported against.  Asynchronous on hip_stream; the caller
 * owns both buffers.  PROPS_EINVAL for a null or misaligned pointer (bytes = 0 is a no-op);
 * PROPS_ETOOBIG beyond (2^24 - 1) x 16 KiB (just under 256 GiB) in one call. */
int props_stream_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

/* ------------------------------------------------------------------ errors */
const char *props_last_error(void);
const char *props_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PROPS_H */
