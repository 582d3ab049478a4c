/*
 * ahr.h -- C ABI of libahr, an MI355X (gfx950) implementation of the signed
 * netlist graph filter at the heart of the area-hint refinement initializer
 * of "Bridging the Initialization Gap: A Co-Optimization Framework for
 * Mixed-Size Global Placement" (arXiv 2511.10073).
 *
 * The method (Section V of the paper):
 *   - a placement instance is a graph G = (V, E) whose nodes are the objects
 *     and whose nets are edges (Section IV, problem statement);
 *   - a fixed macro is split into fixed nodes at its pin sites (Section V,
 *     "Macro pin expansion");
 *   - one virtual node per macro joined by negative edges to the movable
 *     cells inside its footprint (Section V, "Macro virtual node");
 *   - one virtual node per bin joined by signed, density-aware edges to the
 *     movable cells in a detection window (Section V, "Bin virtual node");
 *   - the refinement filter H_r = ((lambda_up I - L_hint)/lambda_up)^k with
 *     lambda_up a Gershgorin bound (Section V, eq. "refine-filter");
 *   - Algorithm 1: T_hint rounds of build / filter / relax (Section V);
 *   - the half-perimeter wirelength that scores a placement.
 *
 * Readings of passages the paper leaves open (net model, signed degree,
 * normalisation, window shape, pinning) are fixed the same way here and in
 * the project's CPU oracle; each is named where it applies below.
 *
 * Conventions for every call:
 *   - All array pointers are DEVICE pointers on the current HIP device unless
 *     marked "host".  The caller owns them; the library never frees them and
 *     keeps no pointer to them after the call returns, except the netlist
 *     arrays a graph handle was built from (those must outlive the handle).
 *   - Signals are row-major [rows][ncols] float32; ncols is 1, 2, 4 or 8.
 *     Columns 2c and 2c+1 are the x and y of placement c.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on it unless documented as synchronous; calls that size
 *     device memory from device-computed counts synchronise the stream.
 *   - Every call returns an ahr_status.  Arguments are validated before any
 *     device work is queued, so an AHR_EINVAL return leaves outputs untouched.
 *     ahr_last_error() returns a message for the calling thread's last error.
 *   - Index ranges are int32: more than 2^31 - 1 nodes, pins or graph entries
 *     give AHR_EUNSUPPORTED.
 *   - Results are deterministic: the same inputs give bit-identical outputs.
 *   - Calls on one graph handle must not overlap (same or different streams).
 */
#ifndef AHR_H
#define AHR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ahr_status;
#define AHR_OK 0
#define AHR_EINVAL (-1)          /* bad argument; nothing was launched        */
#define AHR_ENOMEM (-2)          /* workspace too small, or device allocation failed */
#define AHR_EDEVICE (-3)         /* a HIP call failed                          */
#define AHR_EUNSUPPORTED (-4)    /* valid but outside what this build handles  */

/* node_flags bits */
#define AHR_NODE_FIXED 1u
#define AHR_NODE_MACRO 2u

/* A netlist (Section IV: objects are nodes, nets are hyperedges).
 * Instances are numbered 0..n_inst-1.  A movable standard cell has flags 0;
 * a macro has AHR_NODE_MACRO (plus AHR_NODE_FIXED if fixed); an I/O pin has
 * AHR_NODE_FIXED.  Net e holds pins net_ptr[e] .. net_ptr[e+1]-1. */
typedef struct ahr_netlist {
    int32_t n_inst;
    int32_t n_nets;
    int32_t n_pins;
    int32_t reserved0;          /* must be 0 */
    const int32_t* net_ptr;     /* [n_nets + 1], non-decreasing, net_ptr[0] = 0 */
    const int32_t* pin_node;    /* [n_pins] instance of each pin, in [0, n_inst) */
    const float* pin_off;       /* [n_pins][2] pin offset from the instance centre (may be NULL if n_pins = 0) */
    const float* net_w;         /* [n_nets] net weights, or NULL for all 1 */
    const uint8_t* node_flags;  /* [n_inst] */
    const float* node_size;     /* [n_inst][2] width, height */
    float die[4];               /* host values: xl, yl, xh, yh (xl < xh, yl < yh) */
} ahr_netlist;

/* ahr_hint_params.flags */
#define AHR_EXPAND_MACRO_PINS 1u  /* Section V, macro pin expansion (fixed macros) */
#define AHR_MACRO_HINTS 2u        /* Section V, macro virtual nodes               */
#define AHR_BIN_HINTS 4u          /* Section V, bin virtual nodes                 */
#define AHR_ALL_HINTS 7u
/* Execution order of the filter (performance only; results do not depend on
 * it beyond float32 summation order).  By default the instances follow the
 * Hilbert curve of the first placement the graph sees.  AHR_LAYOUT_NETLIST
 * makes them follow a Cuthill-McKee order of the netlist's
 * instance-to-instance edges instead (graphs with n_inst < 2^22; larger ones
 * keep the Hilbert order); AHR_LAYOUT_AUTO takes that order only where fewer
 * than a quarter of a sample of those edges join rows within n_inst/64 rows
 * (at least 256) of each other in the Hilbert order.  The netlist order costs
 * about 2 ms per graph build at 2.2M cells and cuts the hop's time by about
 * a third where the placement carries no locality (uniformly drawn
 * positions), so it pays where one graph is filtered several times from
 * such a placement.  ahr_graph_info.layout reports the
 * order taken. */
#define AHR_LAYOUT_AUTO 8u
#define AHR_LAYOUT_NETLIST 16u

/* Area-hint parameters (Section V; the refinement block of the paper's
 * parameter table: refine_num_bin_xy, detection_ratio, bin_capacity). */
typedef struct ahr_hint_params {
    int32_t nbx, nby;           /* numBin_x, numBin_y, each in [1, 4096] */
    float detection_ratio;      /* window n = max(1, floor(ratio * numBin)), ratio in [0, 1] */
    float bin_capacity;         /* C in phi_b = 2 sigmoid(mu (D_b - C)) - 1 */
    float mu;                   /* mu > 0 */
    int32_t clique_max;         /* nets with 2 <= p <= clique_max are cliques, larger ones stars; >= 1 */
    uint32_t flags;             /* AHR_EXPAND_MACRO_PINS | AHR_MACRO_HINTS | AHR_BIN_HINTS,
                                   at most one of AHR_LAYOUT_AUTO, AHR_LAYOUT_NETLIST */
    float prune_tau;            /* sparsification (Section IX, "Further speedups"; reading: an edge's
                                   salience is its weight over the cell's baseWeight): bin edges with
                                   exp(-maxRatio) |phi_b| below prune_tau are left out, both directions,
                                   decided in float64; macro edges always stay.  0 keeps every edge;
                                   in [0, 1] */
} ahr_hint_params;

#define AHR_LAMBDA_GERSHGORIN 0
#define AHR_LAMBDA_FIXED 1
#define AHR_MAX_BANDS 4

/* Polynomial filter out = sum_b alpha[b] T^k[b] X with T = I - L/lambda_up
 * (Section V eq. "refine-filter"; a bank of such powers as in Section IV eq.
 * "GiFt filter").  k[b] in [0, 64]; sigma >= 0 is the self-loop weight of
 * Section IV (A_sigma = A + sigma I). */
typedef struct ahr_filter_spec {
    int32_t nbands;             /* 1..AHR_MAX_BANDS */
    int32_t k[AHR_MAX_BANDS];
    float alpha[AHR_MAX_BANDS];
    float sigma;
    int32_t lambda_mode;        /* AHR_LAMBDA_GERSHGORIN or AHR_LAMBDA_FIXED */
    float lambda_fixed;         /* used when lambda_mode == AHR_LAMBDA_FIXED; >= 0 */
} ahr_filter_spec;

/* GiFt's multi-band bank (Section IV eq. "GiFt filter"):
 * H = sum_b alpha[b] Atilde_{sigma[b]}^k[b] with the augmented normalised
 * adjacency Atilde_sigma = D_sigma^-1/2 (A + sigma I) D_sigma^-1/2,
 * D_sigma = D + sigma I (Section IV eq. "GiFt" and the self-loop amendment).
 * The paper's bands are (k, sigma) = (2, 2) high, (2, 4) mid, (4, 4) low. */
typedef struct ahr_gift_spec {
    int32_t nbands;             /* 1..AHR_MAX_BANDS */
    int32_t k[AHR_MAX_BANDS];   /* [0, 64] */
    float alpha[AHR_MAX_BANDS];
    float sigma[AHR_MAX_BANDS]; /* >= 0; bands with equal sigma share one chain of products */
} ahr_gift_spec;

typedef struct ahr_graph ahr_graph;   /* opaque; owns its device memory */

/* Sizes and node ranges of a built graph (host struct).  Canonical node
 * order: instances [0, n_inst); macro pin nodes [first_mpin, first_star)
 * in pin order; star nodes [first_star, first_mvirt) in net order; macro
 * virtual nodes [first_mvirt, first_bvirt) in instance order; bin virtual
 * nodes [first_bvirt, n_tot) row-major by (by, bx). */
typedef struct ahr_graph_info {
    int32_t n_inst, n_tot;
    int32_t first_mpin, first_star, first_mvirt, first_bvirt;
    int32_t nnz_net, nnz_hint;
    int32_t n_hint_cells;       /* movable standard cells that carry hint edges */
    int32_t n_long_rows;        /* rows the filter splits over several workgroups */
    int32_t hint_version;       /* incremented by every hint (re)build */
    int32_t layout;             /* execution order: 0 positions (Hilbert), 1 netlist (Cuthill-McKee) */
    int32_t hop_lanes;          /* the hop's launch shape for this graph under AHR_HOP_AUTO (4 or
                                   AHR_HOP_ROW_BLOCK); 0 until its first filter call */
    int32_t reserved;
    int64_t ws_bytes;           /* the caller's workspace (0: the library's pool) */
    int64_t ws_peak;            /* most of it in use at once so far */
} ahr_graph_info;

/* Host buffers for ahr_graph_export; each pointer may be NULL to skip it.
 * Sizes: net_row_ptr/hint_row_ptr [n_tot+1], net_col/net_q [nnz_net],
 * hint_col/hint_val [nnz_hint], degree/scale [n_tot]. */
typedef struct ahr_graph_host {
    int32_t* net_row_ptr;
    int32_t* net_col;
    int64_t* net_q;             /* netlist weights in units of 2^-32 */
    int32_t* hint_row_ptr;
    int32_t* hint_col;
    float* hint_val;
    double* degree;             /* d_i = sum_j |A_ij| (+ sigma) of the last filter's operator */
    float* scale;               /* s_i = (d_i)^-1/2, 0 for isolated rows */
    float* lambda_up;           /* one value */
} ahr_graph_host;

/* Thread-local message of the last failed call ("" if none). */
const char* ahr_last_error(void);

/* Library version, e.g. "ahr 0.1 gfx950". */
const char* ahr_version(void);

/* Device memory of a graph (two-phase, so that the caller's allocator
 * provides it): an upper bound on the bytes a graph of this netlist and
 * these parameters holds at once through its build and every later call
 * with at most `ncols` columns (ncols in {1, 2, 4, 8}).
 * It counts the netlist's graph entries, star nets and macro pins exactly
 * (one pass over the netlist on `stream`, which it synchronises; 40 bytes of
 * pool memory for the counters) and bounds what the placement decides:
 * hint entries by the detection window and at most four macro footprints
 * holding any one movable standard cell (true when footprints do not
 * overlap), with a 25 % margin for fragmentation.  A graph whose needs
 * exceed its workspace fails with AHR_ENOMEM, its outputs untouched. */
ahr_status ahr_graph_workspace_size(const ahr_netlist* nl, const ahr_hint_params* hp, int32_t ncols,
                                    void* stream, size_t* bytes);

/* Build the graph of a netlist (Section V: macro pin expansion, then the
 * clique/star net model -- reading: weight w/(p-1) per pin pair for
 * 2 <= p <= clique_max, else a star node with w p/(p-1) per spoke -- with
 * parallel edges summed exactly in units of 2^-32) and, if `g` is not
 * NULL, the area hints of the placement held in columns 0 and 1 of `g`
 * ([n_inst][ncols]).  The netlist arrays must stay valid and unchanged
 * while the handle lives.  On success *out receives a handle the caller
 * frees with ahr_graph_destroy.  Synchronises `stream`.
 *   ws, ws_bytes: NULL for the library's stream-ordered pool, or a device
 *   workspace of at least ahr_graph_workspace_size() bytes (for `ncols`
 *   columns, or 8 when `g` is NULL) that every device
 *   allocation of this graph (build and later calls) is carved from; the
 *   caller owns it and may reuse it once the graph is destroyed and its work
 *   on its stream is done.  A workspace below the netlist's fixed arrays
 *   gives AHR_ENOMEM before any device work; below the full bound, after the
 *   counting pass, with nothing built. */
ahr_status ahr_graph_build(const ahr_netlist* nl, const ahr_hint_params* hp,
                           const float* g, int32_t ncols, void* ws, size_t ws_bytes,
                           void* stream, ahr_graph** out);

/* Rebuild the area hints (BuildLap of Algorithm 1: bin densities, phi_b,
 * bin-window and macro-footprint edges) for the placement in columns 0 and
 * 1 of `g` ([n_inst][ncols]).  Synchronises `stream`. */
ahr_status ahr_graph_update_hints(ahr_graph* gr, const float* g, int32_t ncols,
                                  void* stream);

/* Sizes and node ranges (host struct).  The entry counts are read from the
 * device the first time they are asked for after a build or hint update
 * (waiting for the stream the graph's work went to); no other device work. */
ahr_status ahr_graph_get_info(const ahr_graph* gr, ahr_graph_info* info);

/* Copy the graph to host buffers (synchronous; for tests).  Rows are in
 * canonical node order.  Netlist rows list columns in ascending order;
 * virtual rows list their cells grouped by bin (row-major), ascending
 * within a bin -- the order the filter sums them in. */
ahr_status ahr_graph_export(const ahr_graph* gr, ahr_graph_host* dst, void* stream);

/* Free a graph and its device memory.  When all of the graph's work was
 * enqueued on one stream, the memory is released in that stream's order
 * (later work on any stream reuses it only after the graph's work) and the
 * call does not wait; otherwise it synchronises the device.  That stream must
 * still exist when the graph is freed. */
void ahr_graph_destroy(ahr_graph* gr);

/* Apply the polynomial filter of `spec` (Section V eq. "refine-filter";
 * ComputeFilter and the product of Algorithm 1) to `in` ([n_inst][ncols]):
 * the signal is first extended to the added nodes (macro pin node = macro
 * centre + pin offset, star node = mean of its pins, macro virtual node =
 * macro centre, bin virtual node = bin centre), the operator is normalised
 * by absolute degrees d_i = sum_j |A_ij| + sigma (reading for signed
 * graphs), lambda_up is the Gershgorin bound max_i (L_ii + sum_j |L_ij|)
 * or lambda_fixed, and after the whole polynomial every fixed or virtual
 * row is reset to its input.  Writes `out` ([n_inst][ncols]); `in` and
 * `out` must not overlap.  Asynchronous. */
ahr_status ahr_filter(ahr_graph* gr, const ahr_filter_spec* spec,
                      const float* in, float* out, int32_t ncols, void* stream);

/* GSP-based initialization (Section IV, steps 2 and 3): apply the GiFt
 * bank `spec` to `in` ([n_inst][ncols]; movable instances at sampled
 * positions, fixed ones at theirs) on the graph's netlist part, then reset
 * every fixed row to its input; the result is Algorithm 1's g^(0).  The
 * graph must carry no area hints (built with AHR_MACRO_HINTS and
 * AHR_BIN_HINTS off, with a placement for its execution order); the
 * instance graph of Section IV treats macros as points, so
 * AHR_EXPAND_MACRO_PINS is normally off too.  Added star nodes carry the mean
 * of their pins.  in and out must not overlap.  Asynchronous. */
ahr_status ahr_gift(ahr_graph* gr, const ahr_gift_spec* spec, const float* in, float* out, int32_t ncols,
                    void* stream);

/* Algorithm 1 (Section V) on a built graph: for r = 0 .. T_hint-1, rebuild
 * the hints from columns 0 and 1 of g^(r), filter all columns, and relax
 * g^(r+1) = (1 - gamma) g^(r) + gamma g~ on movable rows (fixed rows keep
 * their input).  g0 and out are [n_inst][ncols] and may be the same
 * buffer.  gamma in [0, 1], T_hint >= 0.  Synchronises `stream` once per
 * round (hint sizes). */
ahr_status ahr_graph_refine(ahr_graph* gr, const ahr_filter_spec* spec, const float* g0,
                            int32_t ncols, int32_t T_hint, float gamma, float* out,
                            void* stream);

/* Algorithm 1 end to end, the initializer (Section V; its inputs g^(0), the
 * macros M, the bin capacity C, T_hint and gamma): build the graph of `nl`
 * with `hp` (in the workspace `ws` when it is not NULL, as
 * ahr_graph_build), run ahr_graph_refine, free the graph.  The workspace may
 * be reused once the call's work on `stream` is done. */
ahr_status ahr_refine(const ahr_netlist* nl, const ahr_hint_params* hp, const ahr_filter_spec* spec,
                      const float* g0, int32_t ncols, int32_t T_hint, float gamma, float* out,
                      void* ws, size_t ws_bytes, void* stream);

/* Half-perimeter wirelength of the netlist `nl` (the paper's wirelength
 * score; Section II-B names HPWL as what the WA model approximates) for
 * every placement held in `g` ([n_inst][ncols], ncols 2, 4 or 8): for each
 * column pair c, out[c] = sum over nets of (max - min) pin x + (max - min)
 * pin y, pin position = instance position + pin offset, over the netlist's
 * own pins (no macro pin expansion, no added nodes), accumulated in float64
 * in a fixed order.  `out` is a device array of ncols/2 doubles.  Needs no
 * graph.  Its partial sums come from the library's stream-ordered pool, so
 * calls on different streams may overlap.  Asynchronous. */
ahr_status ahr_hpwl(const ahr_netlist* nl, const float* g, int32_t ncols, double* out, void* stream);

/* ------------------------------------------------------------------------
 * Weighted-average (WA) wirelength and its gradient (Section II-B,
 * "Wirelength model"): the smooth wirelength of the electrostatic global
 * placer the initializer hands its placement to.  For net e and axis x,
 *   xbar+_e = sum_i x_i exp(x_i/gamma) / sum_i exp(x_i/gamma),
 *   xbar-_e = sum_i x_i exp(-x_i/gamma) / sum_i exp(-x_i/gamma),
 * over the netlist's own pins (pin = instance position + pin offset), and
 *   W = sum_e (xbar+_e - xbar-_e) + (ybar+_e - ybar-_e)   (no net weights).
 * Evaluated in float64 (each exponential taken relative to the net's
 * extreme coordinate, which cancels in the ratio).  The gradient of an
 * instance is the sum of its pins' gradients, added exactly in int64 fixed
 * point (2^-40 units; instances with fewer than 2^20 pins), rounded once to
 * float32: deterministic.
 * ------------------------------------------------------------------------ */
typedef struct ahr_wl ahr_wl;          /* opaque: a netlist's instance -> pin index */

/* Index the pins of every instance of `nl` (device arrays, kept by the
 * handle: they must outlive it).  Synchronises `stream`. */
ahr_status ahr_wl_create(const ahr_netlist* nl, void* stream, ahr_wl** out);

/* WA wirelength of every placement in g ([n_inst][ncols], ncols 2, 4 or 8;
 * columns 2c, 2c+1 are placement c): wl (device, ncols/2 doubles) and, if
 * grad is not NULL, dW/dg (device [n_inst][ncols] float32).  gamma > 0.
 * Work buffers come from the library's pool.  Asynchronous. */
ahr_status ahr_wa(ahr_wl* h, const float* g, int32_t ncols, float gamma, double* wl, float* grad, void* stream);
void ahr_wl_destroy(ahr_wl* h);

/* ------------------------------------------------------------------------
 * Macro charge-density models (Section VI, "Macro-Schedule Global
 * Placement"): each macro's footprint carries an iteration-dependent density
 * rho_t(dx, dy) (offsets from its centre, |dx| <= w/2, |dy| <= h/2), and its
 * contribution to bin b is the integral of rho_t over the part of b inside
 * the footprint (the section's closing equation).
 * ------------------------------------------------------------------------ */
#define AHR_CHARGE_GAUSSIAN 0   /* Section VI-A eqs. "Gaussion_eta", "eta_t" (charge redistribution)   */
#define AHR_CHARGE_EXP 1        /* Section VI-B eqs. "exp_sigma", "sigma_t" (restoration, the default) */
#define AHR_CHARGE_LINEAR 2     /* eq. "linear_k", clipped below at 0 (reading)                        */
#define AHR_CHARGE_SIGMOID 3    /* eq. "sigmoid_k"                                                      */

typedef struct ahr_charge_params {
    int32_t model;              /* AHR_CHARGE_* */
    int32_t t, T;               /* iteration t in [0, T], T >= 1 (schedule_iteration) */
    int32_t nbx, nby;           /* bins tiling the die, each in [1, 4096] */
    float sigma_factor;         /* exponential model: sigma(t) = -sigma_factor T ln(1 - t/T); > 0 */
    float k_factor;             /* linear, sigmoid: k(t) = k_factor / tan(pi t / 2T); > 0 */
    float r0, r1;               /* Gaussian Scheme A: edge decay ratio at t = 0 and T, in (0, 1) */
    float beta_min, beta_max;   /* Gaussian Scheme B: normalised FWHM at t = 0 and T, > 0 */
    float alpha0, alpha1;       /* Gaussian blend: smoothstep from alpha0 to alpha1, 0 <= alpha0 < alpha1 <= 1 */
} ahr_charge_params;

/* The model's parameter at iteration t (host, float64): eta, sigma or k.
 * The end points are limits: sigma(0) = 0 and k(0) = +inf (no charge),
 * sigma(T) = +inf and k(T) = 0 (the flat footprint, rho = 1). */
ahr_status ahr_charge_schedule(const ahr_charge_params* cp, double* param);

/* Per bin b (row-major by (by, bx)): bin_mass[b] = the sum over every macro
 * of the netlist (at columns 0 and 1 of `g`, [n_inst][ncols], ncols >= 2) of
 * the integral of its rho_t over bin b inside its footprint, in area units.
 * Footprint parts outside the die fall in no bin.  Float64; the Gaussian by
 * erf differences, the others by fixed Gauss-Legendre rules on panels that
 * follow each integrand's scales (within about 1e-13 of the exact integral
 * relative to the macro area); per-bin sums in 2^-28 fixed point, so the
 * result does not depend on summation order.  bin_mass is a device array of
 * nbx * nby doubles.  Synchronises `stream` once (the pair count). */
ahr_status ahr_macro_charge(const ahr_netlist* nl, const float* g, int32_t ncols, const ahr_charge_params* cp,
                            double* bin_mass, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ahr_hpwl
 * with its partial sums in a fixed library-owned device buffer of
 * ahr_hpwl_noalloc_bytes() bytes (256 KiB) per device, held until the
 * process ends, instead of pool memory.  It calls no allocator.  The buffer
 * holds the partials of any netlist size; ncols above 8 is rejected
 * (AHR_EINVAL).  Every call on a device shares that device's buffer, and
 * each call overwrites it completely before reading it, so calls that
 * overlap in time on one device (on any streams) race and give wrong totals;
 * calls ordered on one stream are safe.  Same result bits as ahr_hpwl.
 * Asynchronous. */
ahr_status ahr_hpwl_noalloc(const ahr_netlist* nl, const float* g, int32_t ncols, double* out, void* stream);
size_t ahr_hpwl_noalloc_bytes(void);

/* ------------------------------------------------------------------------
 * Learned surrogate of the filter (a project addition; the paper has no
 * learned component).  It approximates the polynomial filter of `spec` from
 * the input and three powers of the same operator: for every instance row i
 * and column c,
 *   h_j = (T^j X)[i,c] (j = 0..3, unpinned; h_0 = X), m_c / s_c = mean /
 *   standard deviation of h_3 over movable rows, r_c = root mean square of
 *   h_0 - h_3 over movable rows (a zero s_c or r_c becomes 1),
 *   f = [(h0-h3)/r_c, (h1-h3)/r_c, (h2-h3)/r_c, (h3-m_c)/s_c, log1p(d_i),
 *        hsum_i/d_i, log(s_c/r_c)]
 *   (d_i the absolute degree, hsum_i the signed sum of the row's hint weights),
 *   o = w3 . relu(W2 relu(W1 f + b1) + b2) + b3,
 *   y = beta[0] h0 + beta[1] h1 + beta[2] h2 + beta[3] h3 + r_c o; fixed rows
 *   keep their input.
 * The network is evaluated with bfloat16 operands (features, weights, hidden
 * activations; round to nearest even) and float32 accumulation on the matrix
 * cores.  Parameters are one float32 device vector of AHR_MLP_NPARAM values:
 * W1[64][8] (feature 7 unused), b1[64], W2[64][64], b2[64], w3[64], b3.
 * ------------------------------------------------------------------------ */
#define AHR_MLP_HIDDEN 64
#define AHR_MLP_FEATURES 7
#define AHR_MLP_FEATURE_STRIDE 8
#define AHR_MLP_NPARAM 4801

typedef struct ahr_mlp {
    const float* params;        /* device [AHR_MLP_NPARAM] */
    float beta[4];              /* weights of h0 (the input), h1, h2, h3 */
    int32_t validated;          /* 0: the model missed its validation bound; the plain filter runs */
} ahr_mlp;

/* The learned filter: same operator normalisation as ahr_filter (sigma,
 * lambda from `spec`), three hops, features, MLP.  If model->validated is 0
 * the plain ahr_filter(spec) runs instead and *used_fallback (host, may be
 * NULL) is set to 1, else 0.  in/out [n_inst][ncols], no overlap. */
ahr_status ahr_filter_learned(ahr_graph* gr, const ahr_filter_spec* spec, const ahr_mlp* model,
                              const float* in, float* out, int32_t ncols, int32_t* used_fallback,
                              void* stream);

/* Algorithm 1 (as ahr_refine) with the learned filter in place of the
 * plain one in every round: hints rebuilt from the current placement, the
 * surrogate (3 hops + the per-node network, see ahr_filter_learned) applied,
 * then the relaxation g <- (1 - gamma) g + gamma g~ on movable rows.  An
 * unvalidated model runs the plain filter instead (*used_fallback = 1).  A
 * project addition: the paper's Algorithm 1 uses the filter of Section V. */
ahr_status ahr_refine_learned(ahr_graph* gr, const ahr_filter_spec* spec, const ahr_mlp* model, const float* g0,
                              int32_t ncols, int32_t T_hint, float gamma, float* out, int32_t* used_fallback,
                              void* stream);

/* Training data of the surrogate: for the signal `in` ([n_inst][ncols]),
 * writes feats [n_inst*ncols][AHR_MLP_FEATURE_STRIDE] (instance order, row
 * i*ncols + c), hops [4][n_inst][ncols] (h0, h1, h2, h3) and stats [3][ncols]
 * (m_c, s_c, r_c).  Any output may be NULL. */
ahr_status ahr_filter_features(ahr_graph* gr, const ahr_filter_spec* spec, const float* in, int32_t ncols,
                               float* feats, float* hops, float* stats, void* stream);

/* o[k] = MLP(feats[k]) for n feature rows (stride AHR_MLP_FEATURE_STRIDE),
 * matrix-core evaluation as above. */
ahr_status ahr_mlp_forward(const float* params, const float* feats, int64_t n, float* o, void* stream);

/* Training: *loss (device double, may be NULL) = mean_k (MLP(feats[k]) -
 * target[k])^2 and grad (device [AHR_MLP_NPARAM]) its gradient, float32
 * arithmetic, fixed-order (deterministic) reductions.  rounding = 1: the
 * inference's bfloat16 rounding points (weights, features, hidden
 * activations) with straight-through gradients, as training uses;
 * rounding = 0: float32 operands throughout (for checking the gradient
 * against a float64 reference without rounding).  Other values: AHR_EINVAL. */
ahr_status ahr_mlp_loss_grad(const float* params, const float* feats, const float* target, int64_t n,
                             float* grad, double* loss, int32_t rounding, void* stream);

/* One Adam step (step >= 1) on params with moments m, v (all device
 * [AHR_MLP_NPARAM]). */
ahr_status ahr_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step, float lr,
                        float beta1, float beta2, float eps, void* stream);

/* Return the device memory that freed graphs left in the library's cache
 * to the driver (graph builds reuse cached blocks).  Synchronises on the
 * frees still in flight. */
ahr_status ahr_memory_trim(void);

/* Launch shape of the filter's SpMM hop (process-wide; a batch's own
 * configuration, ahr_batch_set_config / ahr_batch_autotune, overrides it
 * for that batch): lanes_per_row in {1, 2, 4, 8, 16, 32, 64} lanes of a
 * wavefront share one row of up to 128 entries (0 keeps the current
 * value); nontemporal = 1 streams the adjacency with non-temporal loads so
 * the L2 keeps the gathered signal rows (-1 keeps the current value).
 * lanes_per_row = AHR_HOP_ROW_BLOCK selects the row-block form instead:
 * one workgroup per block of consecutive short rows (at most 256 rows and
 * 1151 entries) streams the block's entries with coalesced loads, stages
 * the weighted products in LDS and adds each row's products in entry
 * order.  Each setting is deterministic; settings differ from each other
 * in the last bits only (the summation order of a row changes).
 * lanes_per_row = AHR_HOP_AUTO (the default) picks per graph: 4 lanes where
 * the execution order is local (at least a quarter of a sample of the
 * instance-to-instance entries lie within n_inst/64 rows, at least 256, of
 * their row), else the row-block form, which keeps more of the gathers in
 * flight when most of them miss the caches (at 2.2M cells, 521 against 597
 * us per hop in the order of GiFt's output, 268 against 254 us in a local
 * order).  The first hop of a filter call that forms the Gershgorin bound
 * always uses 4 lanes. */
#define AHR_HOP_ROW_BLOCK 256     /* lanes_per_row value selecting the row-block hop */
#define AHR_HOP_AUTO 1024         /* lanes_per_row value: the shape follows each graph's order */
ahr_status ahr_filter_tune(int32_t lanes_per_row, int32_t nontemporal);
ahr_status ahr_filter_get_tune(int32_t* lanes_per_row, int32_t* nontemporal);

/* ---------------------------------------------------------------------------
 * Batched filter (a project addition; the paper filters one netlist at a
 * time).  Many netlists of uneven size are built once (graph and area hints
 * each, as ahr_graph_build) and laid out as one block-diagonal operator,
 * each block with its own lambda_up; one ahr_batch_filter call then applies
 * the filter bank of ahr_filter (Section V, eq. "refine-filter", banked as
 * in Section IV eq. "GiFt filter") to all of them with one launch per
 * power of T, captured once as a HIP graph and replayed.
 *
 * Signals are the members' instance rows concatenated in member order:
 * member g's rows start at row sum_{h<g} nls[h].n_inst, row-major with
 * ncols columns.  For the same lanes_per_row every member's output is
 * bit-identical to ahr_filter on that member alone (each column's sums run
 * in the same order for every column tile).
 */
typedef struct ahr_batch ahr_batch;    /* opaque; owns its device memory and member graphs */

typedef struct ahr_batch_info {
    int32_t n_graphs;
    int32_t n_inst;             /* instance rows of all members */
    int32_t n_tot;              /* rows of the batched operator */
    int32_t n_long_rows;        /* rows summed by whole workgroups */
    int64_t nnz_net, nnz_hint;  /* entries of the batched netlist and hint lists */
    int32_t n_captured;         /* captured call shapes held (at most 16, least recently used dropped) */
    int32_t reserved;
} ahr_batch_info;

/* Build n member graphs from host arrays nls[n], hps[n] (device pointers
 * inside, owned by the caller and kept) and the concatenated placement pos
 * (device, [sum n_inst][ncols], ncols in {2, 4, 8}; columns 0, 1 are used
 * for the area hints).  Synchronises on `stream`.  EINVAL on a bad member
 * (the message names it) before any device work; EUNSUPPORTED when the
 * batch reaches 2^31 rows or list entries. */
ahr_status ahr_batch_build(const ahr_netlist* nls, const ahr_hint_params* hps, int32_t n, const float* pos,
                           int32_t ncols, void* stream, ahr_batch** out);
ahr_status ahr_batch_get_info(const ahr_batch* b, ahr_batch_info* info);

/* Filter every member: in, out device [sum n_inst][ncols], not
 * overlapping; fixed rows of out = in.  use_graph = 1 replays (capturing on
 * first use) the HIP graph of this (spec, ncols, launch shape, in, out);
 * 0 launches the same kernels directly.  Asynchronous on `stream` once
 * captured (capturing synchronises once).  The member operators are
 * normalised for spec on first use and whenever sigma or lambda_mode
 * change. */
ahr_status ahr_batch_filter(ahr_batch* b, const ahr_filter_spec* spec, const float* in, float* out, int32_t ncols,
                            int32_t use_graph, void* stream);

/* Launch shape for ncols columns: lanes_per_row (power of two in [1, 64] or
 * AHR_HOP_ROW_BLOCK; 0 = the process-wide ahr_filter_tune value, 4 lanes
 * when that is AHR_HOP_AUTO) and col_tile (columns per hop pass: a power of
 * two dividing ncols; 0 = ncols). */
ahr_status ahr_batch_set_config(ahr_batch* b, int32_t ncols, int32_t lanes_per_row, int32_t col_tile);
ahr_status ahr_batch_get_config(const ahr_batch* b, int32_t ncols, int32_t* lanes_per_row, int32_t* col_tile);

/* Time every (lanes_per_row in {1, 2, 4, 8, 16, 32, AHR_HOP_ROW_BLOCK},
 * col_tile dividing ncols) on a library-owned input (captured, warmed, mean
 * of 3 replays), keep the fastest as the batch's configuration for ncols
 * and return it (each output pointer may be NULL).  Synchronises on
 * `stream`. */
ahr_status ahr_batch_autotune(ahr_batch* b, const ahr_filter_spec* spec, int32_t ncols, void* stream,
                              int32_t* lanes_per_row, int32_t* col_tile, float* best_ms);
void ahr_batch_destroy(ahr_batch* b);

/* Per-stage device time, measured with HIP events recorded on the stream
 * each stage runs on (process-wide accumulators). */
typedef struct ahr_profile {
    double build_ms, hints_ms, norm_ms, expand_ms, hop_ms, relax_ms, hpwl_ms;
    int64_t build_calls, hints_calls, norm_calls, expand_calls, hop_launches, relax_calls, hpwl_calls;
    double hop_bytes;           /* algorithmic bytes of every timed hop launch (see ahr_filter) */
    double mlp_ms;              /* learned-filter MLP kernel */
    int64_t mlp_calls;
    double wa_ms;               /* WA wirelength (+ gradient) calls */
    int64_t wa_calls;
    double wa_bytes;            /* their algorithmic bytes (see ahr_wa) */
} ahr_profile;

/* Event timing for subsequent calls: 0 off, 1 every stage and hop launch
 * (two event records each), 2 hop launches only (the least added work, for
 * timing the hop inside a timed run).  AHR_EINVAL for other values. */
ahr_status ahr_profile_enable(int32_t on);

/* Wait for the recorded events and return the accumulated times; reset = 1
 * clears the accumulators.  Synchronises on the recorded events. */
ahr_status ahr_profile_read(ahr_profile* out, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* AHR_H */
