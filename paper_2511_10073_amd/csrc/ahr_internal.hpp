// Internal declarations shared by the libahr translation units.
#pragma once

#include <initializer_list>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/ahr.h"

namespace ahr {

// ---------------------------------------------------------------- errors

struct Error {
    ahr_status code;
    std::string msg;
};

void set_error(ahr_status code, const std::string& msg);
ahr_status fail(ahr_status code, const std::string& msg);

// Throws ahr::Error on a failed HIP call; the C entry points catch it.
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define AHR_HIP(call) ::ahr::hip_check((call), #call, __FILE__, __LINE__)
#define AHR_LAUNCHED(name) ::ahr::hip_check(hipGetLastError(), name, __FILE__, __LINE__)

// ---------------------------------------------------------------- memory

// A caller-provided device workspace that one graph's memory is carved from
// (first fit, 256-byte aligned, free neighbours merged).  While an
// ArenaScope is active on a thread, dev_alloc draws from its arena; dev_free
// returns a block to whichever arena holds its address.  A block freed on
// one stream and taken again on another waits for the first stream.
struct Arena;
Arena* arena_create(void* base, size_t bytes);
void arena_destroy(Arena* a) noexcept;
size_t arena_peak(const Arena* a);
size_t arena_size(const Arena* a);
class ArenaScope {
  public:
    explicit ArenaScope(Arena* a);
    ~ArenaScope();
    ArenaScope(const ArenaScope&) = delete;
    ArenaScope& operator=(const ArenaScope&) = delete;

  private:
    Arena* prev_;
};

// Stream-ordered device allocation from a pool that keeps freed memory (or
// from the active arena, see above).  Blocks may be freed on one stream and
// reused on another.
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);
// Records the events that order the blocks freed since the last call behind
// their streams' work (one per stream).  Every entry point calls it before
// it returns, while its stream is still known to exist.
void flush_frees() noexcept;
// A non-blocking stream per device, at the default priority, for work that
// overlaps the caller's stream (joined to it by events); never destroyed.
hipStream_t side_stream();

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;       // capacity in elements
    void ensure(size_t need, hipStream_t s) {
        if (need <= n && p) return;
        if (p) dev_free(p, s);
        size_t cap = need < 1 ? 1 : need;
        p = static_cast<T*>(dev_alloc(cap * sizeof(T), s));
        n = cap;
    }
    void release(hipStream_t s) {
        if (p) dev_free(p, s);
        p = nullptr;
        n = 0;
    }
};

inline unsigned grid_for(int64_t n, int per_block) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return static_cast<unsigned>(g);
}

// ---------------------------------------------------------------- scan

// out[0..n] = exclusive prefix sums of in[0..n-1] (out[n] = total).
// Integer, so deterministic.  `tmp` must hold scan_tmp_elems(n) int64.
size_t scan_tmp_elems(int64_t n);
void scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s);
// Same, writes int32 (caller checked the total fits).
void scan_i32_to_i32(const int32_t* in, int32_t* out, int64_t n, int64_t* tmp, hipStream_t s);
// int32 scan that returns the exact int64 total (one synchronisation); the
// int32 output is only meaningful when the total is below 2^31.
int64_t scan_i32_checked(const int32_t* in, int32_t* out, int64_t n, int64_t* tmp, hipStream_t s);
// The same scan without reading its total: returns the device address of the
// int64 total (valid until tmp is reused), for a later combined read.
const int64_t* scan_i32_total(const int32_t* in, int32_t* out, int64_t n, int64_t* tmp, hipStream_t s);

// list[rank[i]] = i for every i with flags[i] != 0 (rank = exclusive scan of flags).
void list_rows(const int32_t* flags, const int32_t* rank, int32_t n, int32_t* list, hipStream_t s);
// p[0..n) = v
void fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// host[k] = *src[k] for up to 8 device int32 scalars, with one synchronisation
void read_scalars(const std::vector<const int32_t*>& src, int32_t* host, hipStream_t s);
// Device scalars of 4 (wide = 0) or 8 (wide = 1) bytes, read in one synchronisation.
struct DevWord {
    const void* p;
    int wide;
};
void read_words(std::initializer_list<DevWord> src, int64_t* out, hipStream_t s);
// The same read split in two, so that work queued between the halves runs
// while the host waits: read_scalars_begin gathers up to 8 int32 values on
// stream s into the device's pinned words (a second set, kept apart from
// the synchronous reads) and records an event; read_scalars_end waits for
// that event alone and copies the values out.  One read in flight per
// device and host thread.
void read_scalars_begin(const std::vector<const int32_t*>& src, hipStream_t s);
void read_scalars_end(int32_t* host, int n);
// One device scalar (synchronises the stream).
int32_t read_i32(const int32_t* src, hipStream_t s);
int64_t read_i64(const int64_t* src, hipStream_t s);
double read_f64(const double* src, hipStream_t s);

// ---------------------------------------------------------------- profiling

enum Stage { kStageBuild, kStageHints, kStageNorm, kStageExpand, kStageHop, kStageRelax, kStageHpwl, kStageMlp,
             kStageWa, kStageCount };

bool profiling();
// While set (on this thread), ProfScope records nothing: used around HIP
// graph capture, where event records would become graph nodes.
void set_capture(bool on);

// An event pair for one kernel launched with hipExtLaunchKernelGGL: the
// launch binds the events to the kernel's own start and end, so no marker
// packet sits between the kernels.  False (both null) when stage st is not
// being timed; else hand the pair to prof_kernel_done after the launch.
bool prof_kernel_events(Stage st, hipEvent_t* start, hipEvent_t* stop);
void prof_kernel_done(Stage st, hipEvent_t start, hipEvent_t stop, double bytes);

// Records an event pair around its lifetime on stream s when profiling is on.
class ProfScope {
  public:
    ProfScope(Stage st, hipStream_t s, double bytes = 0.0);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

  private:
    int stage_;
    hipStream_t s_;
    double bytes_;
    void* a_ = nullptr;
    bool live_ = false;
};

// ---------------------------------------------------------------- graph

// Rows with more entries than kLongRow are summed by whole workgroups, in
// chunks of kChunk entries; the other rows are grouped into row blocks of
// consecutive rows (at most kRbRows rows and kRbEntries + kLongRow
// entries, never across a long row or the instance boundary) for the
// LDS-staged hop.
constexpr int kLongRow = 128;
constexpr int kChunk = 2048;
constexpr int kRbRows = 256;
constexpr int kRbEntries = 1024;
// Star nodes are averaged over their pins by their row's thread up to
// kStarInline pins, by kStarLanes lanes up to kStarMid pins, and by a whole
// workgroup above (listed per graph in big_stars).
constexpr int kStarInline = 8;
constexpr int kStarMid = 256;
constexpr int kStarLanes = 8;

struct RowClasses {
    DevBuf<int32_t> long_rows;    // rows split over chunks, ascending
    DevBuf<int32_t> long_chunk0;  // [n_long+1] first chunk of each long row
    DevBuf<int32_t> chunk_row;    // [n_chunks] long-row index of each chunk
    DevBuf<double> partial;       // [n_chunks * 8]
    DevBuf<int4> rb;              // [2 n_rb] row blocks: (r0, r1, net_lo, net_hi), (hint_lo, hint_hi, -, -)
    int32_t n_long = 0, n_long_inst = 0;      // long rows, those below n_inst
    int32_t n_chunks = 0, n_chunks_inst = 0;  // chunks, those of long rows below n_inst
    int32_t n_rb = 0, n_rb_inst = 0;          // row blocks, those below n_inst
    int32_t has_rb = 0;                       // row blocks built (on first use of the row-block hop)
    int64_t nnz_inst = 0;                     // entries of rows below n_inst (netlist + hints)
    int64_t nnz_net_all = 0, nnz_hint_all = 0; // entries of all rows
    void release(hipStream_t s) {
        long_rows.release(s);
        long_chunk0.release(s);
        chunk_row.release(s);
        partial.release(s);
        rb.release(s);
    }
};

struct Graph {
    Arena* arena = nullptr;    // the caller's workspace all device memory comes from (null: the pool)
    ahr_netlist nl;            // caller's device arrays (kept)
    ahr_hint_params hp;
    int32_t n_inst = 0, n_mpin = 0, n_star = 0, n_macro = 0, n_bins = 0;
    int32_t first_mpin = 0, first_star = 0, first_mvirt = 0, first_bvirt = 0, n_tot = 0;
    // entry counts; -1 while not read yet (arrays are sized by a bound, the
    // counts ride along with later reads: hint_count / net_count read them)
    mutable int32_t nnz_net = 0, nnz_hint = 0;
    int32_t nnz_cap = 0;        // capacity of the netlist entry arrays (>= nnz_net)
    int32_t n_hint_cells = 0;
    int32_t hint_version = 0;
    int32_t has_hints = 0;
    int device = 0;

    // The streams the graph's work was enqueued on: while there is one, the
    // destructor releases the memory in that stream's order and does not
    // wait for the device.
    mutable hipStream_t work_stream = nullptr;
    mutable int stream_uses = 0;   // 0 none, 1 one stream, 2 several
    void use_stream(hipStream_t s) const {
        if (stream_uses == 0) {
            work_stream = s;
            stream_uses = 1;
        } else if (s != work_stream) {
            stream_uses = 2;
        }
    }

    // netlist part (fixed for the life of the handle)
    DevBuf<int32_t> pin_node_x;   // [n_pins] pin node after macro pin expansion
    DevBuf<int32_t> mpin_owner;   // [n_mpin]
    DevBuf<int32_t> mpin_pin;     // [n_mpin]
    DevBuf<int32_t> star_net;     // [n_star]
    DevBuf<int32_t> macro_ids;    // [n_macro] instance id of each macro (instance order)
    // merged netlist rows in node order, in place: row r holds net_len[r]
    // entries from slot net_off[r] (columns ascending); slots up to the next
    // row's offset are unused (parallel edges merged away)
    DevBuf<int64_t> net_off;      // [n_tot+1]
    DevBuf<int32_t> net_len;      // [n_tot]
    DevBuf<int32_t> net_col;      // [nnz_cap]
    DevBuf<int64_t> net_q;        // [nnz_cap]
    DevBuf<int64_t> qdeg;         // [n_tot]
    DevBuf<double> base_w;        // [n_inst] baseWeight
    DevBuf<int32_t> big_nets;     // nets with more than a wave's worth of pins (HPWL)
    int32_t n_big_nets = 0;
    DevBuf<int32_t> big_stars;    // star indices (0-based) of nets with more than kStarMid pins
    int32_t n_big_stars = 0;

    // hint part (per placement)
    DevBuf<int32_t> cell_bin;     // [n_inst] by execution row: bin of a hint cell, -1 otherwise
    DevBuf<int32_t> bin_start;    // [n_bins+1]
    DevBuf<int32_t> bin_cells;    // [n_hint_cells] execution rows of hint cells by bin, ascending
    DevBuf<int64_t> bin_area_q;   // [n_bins] fixed-point area (2^-28 units)
    DevBuf<int64_t> macro_area_q; // [n_bins] the macros' part of bin_area_q (kept for the next round)
    DevBuf<double> phi;           // [n_bins]
    DevBuf<int32_t> bm_start;     // [n_bins+1] macros whose bin span covers a bin
    DevBuf<int32_t> bm_list;
    DevBuf<int4> macro_span;      // [n_macro] bin span bx0, by0, bx1, by1 of the cells it can hold
    DevBuf<float4> macro_rect;    // [n_macro] cx, cy, w/2, h/2 (float32)
    DevBuf<int32_t> hint_cnt;     // [n_tot]
    DevBuf<int32_t> nmac, nwin;   // [n_inst] per execution row: macros holding the cell, window size
    DevBuf<int32_t> pair_off;     // [n_inst+1] first (cell, macro) pair of each row
    DevBuf<int32_t> pair_row, pair_mac;
    DevBuf<int32_t> mlist, mstart; // pairs grouped by macro
    DevBuf<int32_t> bin_rank;     // [n_inst] position of a hint cell in bin_cells
    DevBuf<int32_t> wpre;         // [n_bins * window slots] offsets of the slots in bin rows
    DevBuf<unsigned long long> keep_mask;  // [n_inst] per execution row: window slots whose bin edge is kept
    DevBuf<int32_t> kept;         // [n_bins * window slots] cells of a bin keeping the edge to each window slot
    DevBuf<int64_t> xcell;        // [n_inst] per execution row: cell area (2^-28 units) * 4 + cell class
    DevBuf<double> xbase_w;       // [n_inst] per execution row: baseWeight
    DevBuf<float2> xpos;          // [n_inst] per execution row: the current placement's (x, y)
    DevBuf<double> xhabs;         // [n_inst] per execution row: sum of |hint weight| (hint_version habs_version)
    DevBuf<float> xhsg;           // [n_inst] per execution row: signed sum of the hint weights
    int32_t habs_version = -1;
    DevBuf<double> gmax;          // first-hop Gershgorin maxima (per workgroup, then per long row)
    int32_t has_xcell = 0;
    int32_t n_movable_macro = 0;  // macros without AHR_NODE_FIXED
    int32_t macro_cache = 0;      // macro_rect/_span, bm_start/_list and macro_area_q hold the fixed macros' values

    // execution layout: instance, macro pin and star rows each in spatial
    // order inside their id range (perm: exec -> id); virtual rows unmoved
    int32_t has_layout = 0;
    int32_t layout_netlist = 0;   // the instances took the netlist (Cuthill-McKee) order
    // locality of the execution order (set with the layout, read with the
    // first row classes): 1 local, 0 not, -1 not read yet
    int32_t hop_local = -1;
    DevBuf<int64_t> loc_part;               // [2 per workgroup] sampled entries near their row, all sampled
    DevBuf<int32_t> loc_flag;               // [1] the verdict on the device
    DevBuf<int32_t> perm, iperm;  // [n_tot]: identity on the virtual rows
    DevBuf<int4> xmpin;           // [n_mpin] per execution macro pin row: owner, offset x, y (float bits)
    DevBuf<int32_t> xstar_net;    // [n_star] per execution star row: its net
    DevBuf<int32_t> xnet_rp;      // [n_tot+1]
    DevBuf<int2> xnet_ent;        // [nnz_net]: read it through net_entries()
    // The copy into xnet_ent runs on the device's side stream: xnet_fork
    // orders it after the layout, xnet_ready is recorded after it.
    // xnet_wait_stream is the last stream made to wait for it (if xnet_waited).
    hipEvent_t xnet_fork = nullptr, xnet_ready = nullptr;
    mutable hipStream_t xnet_wait_stream = nullptr;
    mutable int32_t xnet_waited = 0;
    DevBuf<int64_t> xqdeg;        // [n_tot]
    DevBuf<int32_t> xhint_rp;     // [n_tot+1] hint rows, execution order
    DevBuf<int2> xhint_ent;       // [nnz_hint] (column, float bits of the weight)
    DevBuf<int32_t> lay_start;    // scratch

    // operator (per hint version and sigma), rows in execution order
    DevBuf<double> deg;           // [n_tot]
    DevBuf<float> scale;          // [n_tot]
    DevBuf<float> hsum;           // [n_tot] signed sum of the row's hint weights
    DevBuf<double> lam;           // [1] lambda_up
    double lam_host = 0.0;
    int32_t norm_version = -1;
    float norm_sigma = -1.f;
    int32_t norm_mode = -1;
    float norm_fixed = -1.f;

    DevBuf<float2> coef;          // [n_tot] hop coefficients (cr, kr) of each row (see hop_coef)

    // row classes for the filter
    RowClasses rc;
    int32_t rows_version = -1;

    // filter work buffers
    DevBuf<float> z0, z1, acc;    // [n_tot * C]
    DevBuf<float> zpk;            // first-hop records [n_tot][2, 4 or 8]: z, then the row scale
    DevBuf<float> zh[3];          // [n_tot * C] hops 1..3 of the learned path (scaled coordinates)
    DevBuf<float> ga, gb, gt;     // [n_inst * C] refinement rounds

    // scratch
    DevBuf<int64_t> scan_tmp;
    DevBuf<int32_t> i32a, i32b;
    DevBuf<int64_t> i64a;
    DevBuf<int32_t> counter;      // small device counters

    ~Graph();
};

// workspace.hip: an upper bound on a graph's device memory (one counting
// pass over the netlist on s, synchronised), and the part of it known from
// the sizes alone
size_t graph_workspace_bytes(const ahr_netlist& nl, const ahr_hint_params& hp, int32_t ncols, hipStream_t s);
size_t graph_workspace_floor(const ahr_netlist& nl, int32_t ncols);
// netlist_build.hip
void build_netlist(Graph& g, hipStream_t s);
// Stable bucket sort: list = indices i in [0, n) with key[i] >= 0, grouped by
// key, ascending within a key; start[k] = first position of key k
// (start[nkeys] = count).  nkeys <= 16384.  list holds n entries.  Returns
// the count when read_total (one synchronisation), else -1.
int32_t bucket_sort(Graph& g, const int32_t* key, int32_t n, int nkeys, DevBuf<int32_t>& list,
                    DevBuf<int32_t>& start, hipStream_t s, bool read_total = true);
// The same with its scratch given (i32a, i32b, scan_tmp: grown as needed).
int32_t bucket_sort(const int32_t* key, int32_t n, int nkeys, DevBuf<int32_t>& list, DevBuf<int32_t>& start,
                    DevBuf<int32_t>& i32a, DevBuf<int32_t>& i32b, DevBuf<int64_t>& scan_tmp, hipStream_t s,
                    bool read_total = true);
// Exact entry counts of g, read from its row pointers when not known yet.
int32_t net_count(const Graph& g, hipStream_t s);
int32_t hint_count(const Graph& g, hipStream_t s);
// layout.hip: the execution order of the instance, macro pin and star rows
// (spatial) and the permuted copy of the netlist rows the filter streams
void set_layout(Graph& g, const float* pos, int32_t ncols, hipStream_t s);
// The execution-order netlist entries, with stream s ordered after their copy.
const int2* net_entries(const Graph& g, hipStream_t s);
// hints.hip
// macros_unchanged: the macros sit where the previous call on this graph
// put them (the rounds of Algorithm 1 after the first, whose relaxation
// keeps fixed rows); with every macro fixed, their footprints, per-bin
// areas and bin lists are then reused.
void build_hints(Graph& g, const float* pos, int32_t ncols, hipStream_t s, bool macros_unchanged = false);
// filter.hip
void normalise(Graph& g, const ahr_filter_spec& spec, hipStream_t s);
void run_filter(Graph& g, const ahr_filter_spec& spec, const float* in, float* out,
                int32_t ncols, hipStream_t s);
void relax(Graph& g, const float* gcur, const float* gt, float* gnext, int32_t ncols,
           float gamma, hipStream_t s);
// normalise + the unpinned chain T X, T^2 X, T^3 X into g.zh (scaled coordinates)
void run_hops(Graph& g, const ahr_filter_spec& spec, const float* in, int32_t ncols, hipStream_t s);
// gift.hip: the GiFt bank on the graph (no area hints), fixed rows reset
void run_gift(Graph& g, const ahr_gift_spec& spec, const float* in, float* out, int32_t ncols, hipStream_t s);
// charge.hip: the model parameter at iteration t; per-bin masses of every macro
double charge_schedule(const ahr_charge_params& cp);
void run_macro_charge(const ahr_netlist& nl, const float* pos, int32_t ncols, const ahr_charge_params& cp,
                      double* out, hipStream_t s);
// hpwl.hip: run_hpwl draws its partial sums from the pool; hpwl_launch
// takes a buffer of hpwl_partial_elems() doubles (enough for any netlist)
void run_hpwl(const ahr_netlist& nl, const float* pos, int32_t ncols, double* out, hipStream_t s);
void hpwl_launch(const ahr_netlist& nl, const float* pos, int32_t ncols, double* out, double* partial,
                 hipStream_t s);
size_t hpwl_partial_elems();
// mlp.hip
void run_learned(Graph& g, const ahr_filter_spec& spec, const float* params, const float beta[4], const float* in,
                 float* out, int32_t ncols, float* feats, float* hops, float* stats, hipStream_t s);
void mlp_forward(const float* params, const float* feats, int64_t n, float* o, hipStream_t s);
void mlp_loss_grad(const float* params, const float* feats, const float* target, int64_t n, float* grad,
                   double* loss, bool rounding, hipStream_t s);
void mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step, float lr, float b1, float b2,
              float eps, hipStream_t s);

// ---------------------------------------------------------------- filter chain

// Coefficients of one hop in scaled coordinates (Section V, eq.
// "refine-filter" with T = I - L / lambda_up):
//   z'_i = cr_i z_i + kr_i sum_j A_ij z_j,
//   cr_i = 1 - (nz_i - sigma s_i^2) / lambda,  kr_i = s_i^2 / lambda,
// evaluated in float64 and rounded once; T = I when lambda = 0.
__host__ __device__ inline double fmax_d(double a, double b) { return a > b ? a : b; }
__host__ __device__ inline double fmin_d(double a, double b) { return a < b ? a : b; }

__host__ __device__ inline void hop_coef(float s, double lam, double sigma, float& cr, float& kr) {
    cr = 1.f;
    kr = 0.f;
    if (lam > 0) {
        double sd = s;
        cr = static_cast<float>(1.0 - ((s > 0 ? 1.0 : 0.0) - sigma * sd * sd) / lam);
        kr = static_cast<float>(sd * sd / lam);
    }
}

// Signal expansion of one graph: instance rows from the caller's signal,
// macro pin nodes (macro centre + pin offset), star nodes (mean of their
// pins), macro and bin virtual nodes (macro and bin centres), scaled by s.
// Local row r lands in z row  r < n_inst ? row_inst0 + r : row_aux0 + r - n_inst,
// and z is stored as C/ct column tiles [tile][rows][ct] tile_stride apart.
struct ExpandArgs {
    const float* in;          // [n_inst][C], instance order (in_base + in_off in batched launches)
    int64_t in_off;
    const int32_t* perm;      // execution row -> node (instances, macro pins, stars)
    const int32_t* iperm;     // node -> execution row (instances, macro pins, stars)
    const int4* xmpin;        // per execution macro pin row: owner instance, pin offset x, y (float bits)
    const int32_t* xstar_net; // per execution star row: its net
    const float* scale;
    float* z0;
    float* zpk;               // or, when set, first-hop records: z then the row scale (replaces z0)
    float* acc;               // band at k = 0
    float alpha0;
    int32_t band0;
    int32_t n_inst, first_mpin, first_star, first_mvirt, first_bvirt, n_tot;
    int32_t row_inst0, row_aux0;
    int32_t ct;
    int64_t tile_stride;
    const int32_t* mpin_owner;
    const int32_t* mpin_pin;
    const float* pin_off;
    const int32_t* star_net;
    const int32_t* net_ptr;
    const int32_t* pin_node;
    const int32_t* pin_node_x;
    const int32_t* macro_ids;
    int32_t nbx;
    double xl, yl, bw, bh;
};

// The rows of one operator as the hop chain sees them (one graph, or many
// graphs concatenated block-diagonally).
struct ChainView {
    const int32_t* net_rp;
    const int2* net_ent;
    const int32_t* hint_rp;
    const int2* hint_ent;
    const float* scale;
    const float2* coef;       // per-row (cr, kr), or null: from *lam
    const double* lam;
    double sigma;
    const uint8_t* flags;     // instance flags, instance order
    const int32_t* perm;      // execution row -> instance
    const int32_t* long_rows;
    const int32_t* chunk_row;
    const int32_t* chunk0;
    double* partial;
    const int4* rb;
    int32_t n_tot, n_inst, n_long, n_long_inst, n_chunks, n_chunks_inst, n_rb, n_rb_inst;
    int64_t nnz_inst, nnz_all;
    float* z0;
    float* z1;
    float* acc;
};

// Row classes of an operator with rows [0, N), instance rows first: the
// long rows (more than kLongRow entries) with their chunks and a
// partial-sum buffer for C <= 8 columns.  Resets the row blocks.
void row_classes(const int32_t* net_rp, const int32_t* hint_rp, int32_t N, int32_t n_inst, RowClasses& rc,
                 DevBuf<int64_t>& scan_tmp, hipStream_t s);
// The row blocks of the short rows (for the row-block hop), if not built.
void row_blocks(const int32_t* net_rp, const int32_t* hint_rp, int32_t N, int32_t n_inst, RowClasses& rc,
                DevBuf<int64_t>& scan_tmp, hipStream_t s);
// Hop coefficients (cr, kr) of rows [0, n) from scale and lambda (device).
void hop_coefs(int32_t n, const float* scale, const double* lam, double sigma, float2* coef, hipStream_t s);
// The expansion descriptor of graph g (in, z0, acc, bands and the row
// placement are filled in by the caller).
ExpandArgs expand_args(const Graph& g);
// Expansion of many graphs in two launches: descriptors d[0..ng) on the
// device; blk0[g] the first row workgroup of graph g (n_blocks in all),
// sfirst[g] the first star of graph g (n_star stars in all); big_stars the
// batch star indices of the stars with more than kStarMid pins.
void expand_batch(const ExpandArgs* d, const int32_t* blk0, int32_t n_blocks, const int32_t* sfirst,
                  int32_t n_star, const int32_t* big_stars, int32_t n_big_stars, int32_t ng, const float* in,
                  int32_t ncols, hipStream_t s);
// Hops 1..k_max of the filter bank on an expanded signal (z0 and, for a
// band at k = 0, acc hold it), with lanes per short row and column tiles of
// ct columns; the last hop writes out (instance order, fixed rows = in).
void run_chain(const ChainView& v, const ahr_filter_spec& spec, const float* in, float* out, int32_t ncols,
               int lanes, int ct, hipStream_t s);
int32_t spec_kmax(const ahr_filter_spec& spec, float* alpha_sum);

}  // namespace ahr
