// Batched filter over many netlists (a project addition: the paper filters
// one netlist at a time).  The operators of the member graphs (Section V,
// eq. "refine-filter", each with its own lambda_up) are laid out as one
// block-diagonal operator:
//   rows [0, sum n_inst)         the instance rows of graph 0, 1, ... (execution order each),
//   rows [sum n_inst, n_tot)     the auxiliary rows (macro pins, stars, virtual nodes) of graph 0, 1, ...
// so the last hop of the bank still covers one contiguous prefix.  Each
// row carries its own graph's hop coefficients (cr, kr), so the hop kernels
// run the whole batch in one launch per power.  The expansion and all hops
// of a call are captured once as a HIP graph and replayed; the lanes per
// row and the column tile are chosen per column count by timing every
// candidate.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ahr_internal.hpp"
#include "device_util.hpp"

namespace ahr {

extern int g_hop_lanes;

namespace {

constexpr int kBT = 256;

__device__ __forceinline__ int64_t batch_row(int32_t r, int32_t n_inst, int32_t inst0, int32_t aux0) {
    return r < n_inst ? static_cast<int64_t>(inst0) + r : static_cast<int64_t>(aux0) + (r - n_inst);
}

__global__ void k_batch_row_lens(int32_t n, int32_t n_inst, int32_t inst0, int32_t aux0, const int32_t* __restrict__ rp,
                                 int32_t* __restrict__ len) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (r >= n) return;
    len[batch_row(static_cast<int32_t>(r), n_inst, inst0, aux0)] = rp[r + 1] - rp[r];
}

// One wave per row: copy its entries, columns mapped to batch rows.
__global__ void k_batch_copy_rows(int32_t n, int32_t n_inst, int32_t inst0, int32_t aux0, const int32_t* __restrict__ rp,
                                  const int2* __restrict__ ent, const int32_t* __restrict__ brp, int2* __restrict__ bent) {
    int64_t r = (static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x) / kWave;
    if (r >= n) return;
    const int l = lane_id();
    const int k0 = rp[r], len = rp[r + 1] - k0;
    const int o = brp[batch_row(static_cast<int32_t>(r), n_inst, inst0, aux0)];
    for (int k = l; k < len; k += kWave) {
        int2 e = ent[k0 + k];
        e.x = static_cast<int32_t>(batch_row(e.x, n_inst, inst0, aux0));
        bent[o + k] = e;
    }
}

// Instance rows: batch execution row -> batch instance, and the instance flags.
__global__ void k_batch_inst(int32_t n_inst, int32_t inst0, const int32_t* __restrict__ perm,
                             const uint8_t* __restrict__ flags, int32_t* __restrict__ bperm, uint8_t* __restrict__ bflags) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (i >= n_inst) return;
    bperm[inst0 + i] = inst0 + perm[i];
    bflags[inst0 + i] = flags[i];
}

// Scale and hop coefficients of graph g's rows, with g's lambda_up.
__global__ void k_batch_op(int32_t n, int32_t n_inst, int32_t inst0, int32_t aux0, const float* __restrict__ scale,
                           const double* __restrict__ lam, double sigma, float* __restrict__ bscale,
                           float2* __restrict__ bcoef) {
    int64_t r = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (r >= n) return;
    const int64_t br = batch_row(static_cast<int32_t>(r), n_inst, inst0, aux0);
    const float s = scale[r];
    float cr, kr;
    hop_coef(s, *lam, sigma, cr, kr);
    bscale[br] = s;
    bcoef[br] = make_float2(cr, kr);
}

// K = 0: out = (sum alpha) X on movable rows, X on fixed rows.
__global__ void k_batch_identity(int64_t n, int32_t C, const uint8_t* __restrict__ flags, const float* __restrict__ in,
                                 float* __restrict__ out, float alpha_sum) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (i >= n) return;
    float v = in[i];
    out[i] = (flags[i / C] & AHR_NODE_FIXED) ? v : alpha_sum * v;
}

// Deterministic timing input for the tuner.
__global__ void k_batch_pattern(int64_t n, float* __restrict__ p) {
    int64_t i = static_cast<int64_t>(blockIdx.x) * kBT + threadIdx.x;
    if (i >= n) return;
    uint32_t h = static_cast<uint32_t>(i) * 2654435761u;
    p[i] = static_cast<float>(h >> 8) * 0x1p-24f * 1000.f;
}

bool same_spec(const ahr_filter_spec& a, const ahr_filter_spec& b) {
    if (a.nbands != b.nbands || a.sigma != b.sigma || a.lambda_mode != b.lambda_mode || a.lambda_fixed != b.lambda_fixed)
        return false;
    for (int i = 0; i < a.nbands; ++i)
        if (a.k[i] != b.k[i] || a.alpha[i] != b.alpha[i]) return false;
    return true;
}

}  // namespace

// One captured call: expansion + hops for fixed (spec, C, lanes, tile,
// in, out, work buffers).
struct Captured {
    ahr_filter_spec spec;
    int32_t C = 0, lanes = 0, ct = 0;
    const float* in = nullptr;
    float* out = nullptr;
    const float* z0 = nullptr;
    hipGraphExec_t exec = nullptr;
    DevBuf<ExpandArgs> desc;
    std::vector<ExpandArgs> host_desc;
    uint64_t used = 0;
};

struct Batch {
    std::vector<Graph*> g;
    std::vector<int32_t> inst0, aux0;     // first batch row of each graph's instance / auxiliary rows
    int32_t n_inst = 0, n_tot = 0;
    int64_t nnz_net = 0, nnz_hint = 0;
    int device = 0;

    DevBuf<int32_t> net_rp, hint_rp;
    DevBuf<int2> net_ent, hint_ent;
    DevBuf<int32_t> perm;
    DevBuf<uint8_t> flags;
    DevBuf<float> scale;
    DevBuf<float2> coef;
    std::vector<int32_t> op_version;
    ahr_filter_spec op_spec;
    bool op_valid = false;

    RowClasses rc;

    DevBuf<int32_t> blk0, sblk0;          // first expansion workgroup of each graph's rows; first star of each graph
    int32_t n_blocks = 0, n_star_blocks = 0;   // row workgroups, stars
    DevBuf<int32_t> big_stars;            // batch star indices of the stars with more than kStarMid pins
    int32_t n_big_stars = 0;

    DevBuf<float> z0, z1, acc;
    DevBuf<int64_t> scan_tmp;
    DevBuf<ExpandArgs> eager_desc;
    std::vector<ExpandArgs> eager_host;

    int32_t lanes[9] = {0}, ct[9] = {0};  // per column count; 0: default
    std::vector<Captured*> cache;
    uint64_t clock = 0;
    hipStream_t cap_stream = nullptr;     // capture only (the caller's stream may be the legacy default stream)

    ~Batch();
};

namespace {

constexpr size_t kCacheMax = 16;

void drop(Captured* c, hipStream_t s) {
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    c->desc.release(s);
    delete c;
}

ChainView batch_view(Batch& b, const ahr_filter_spec& spec) {
    ChainView v;
    v.net_rp = b.net_rp.p;
    v.net_ent = b.net_ent.p;
    v.hint_rp = b.hint_rp.p;
    v.hint_ent = b.hint_ent.p;
    v.scale = b.scale.p;
    v.coef = b.coef.p;
    v.lam = nullptr;
    v.sigma = spec.sigma;
    v.flags = b.flags.p;
    v.perm = b.perm.p;
    v.long_rows = b.rc.long_rows.p;
    v.chunk_row = b.rc.chunk_row.p;
    v.chunk0 = b.rc.long_chunk0.p;
    v.partial = b.rc.partial.p;
    v.rb = b.rc.rb.p;
    v.n_tot = b.n_tot;
    v.n_inst = b.n_inst;
    v.n_long = b.rc.n_long;
    v.n_long_inst = b.rc.n_long_inst;
    v.n_chunks = b.rc.n_chunks;
    v.n_chunks_inst = b.rc.n_chunks_inst;
    v.n_rb = b.rc.n_rb;
    v.n_rb_inst = b.rc.n_rb_inst;
    v.nnz_inst = b.rc.nnz_inst;
    v.nnz_all = b.nnz_net + b.nnz_hint;
    v.z0 = b.z0.p;
    v.z1 = b.z1.p;
    v.acc = b.acc.p;
    return v;
}

// Expansion descriptors of every graph for one call shape.
std::vector<ExpandArgs> descriptors(Batch& b, const ahr_filter_spec& spec, int32_t C, int32_t ct) {
    bool b0 = false;
    float a0 = 0.f;
    for (int i = 0; i < spec.nbands; ++i)
        if (spec.k[i] == 0) {
            a0 += spec.alpha[i];
            b0 = true;
        }
    std::vector<ExpandArgs> d(b.g.size());
    for (size_t i = 0; i < b.g.size(); ++i) {
        ExpandArgs e = expand_args(*b.g[i]);
        e.in_off = static_cast<int64_t>(b.inst0[i]) * C;
        e.z0 = b.z0.p;
        e.acc = b.acc.p;
        e.alpha0 = a0;
        e.band0 = b0 ? 1 : 0;
        e.row_inst0 = b.inst0[i];
        e.row_aux0 = b.aux0[i];
        e.ct = ct;
        e.tile_stride = static_cast<int64_t>(b.n_tot) * ct;
        d[i] = e;
    }
    return d;
}

// Per-graph normalisation (cached per graph) and the batch's row scale and
// coefficients when any of them changed.
void ensure_operator(Batch& b, const ahr_filter_spec& spec, hipStream_t s) {
    bool stale = !b.op_valid || b.op_spec.sigma != spec.sigma || b.op_spec.lambda_mode != spec.lambda_mode ||
                 b.op_spec.lambda_fixed != spec.lambda_fixed;
    for (size_t i = 0; i < b.g.size(); ++i) {
        normalise(*b.g[i], spec, s);
        stale = stale || b.op_version[i] != b.g[i]->norm_version;
    }
    if (!stale) return;
    for (size_t i = 0; i < b.g.size(); ++i) {
        Graph& g = *b.g[i];
        hipLaunchKernelGGL(k_batch_op, dim3(grid_for(g.n_tot, kBT)), dim3(kBT), 0, s, g.n_tot, g.n_inst, b.inst0[i],
                           b.aux0[i], g.scale.p, g.lam.p, static_cast<double>(spec.sigma), b.scale.p, b.coef.p);
        AHR_LAUNCHED("k_batch_op");
        b.op_version[i] = g.norm_version;
    }
    b.op_spec = spec;
    b.op_valid = true;
}

void enqueue(Batch& b, const ExpandArgs* desc, const ahr_filter_spec& spec, const float* in, float* out, int32_t C,
             int lanes, int ct, hipStream_t s) {
    expand_batch(desc, b.blk0.p, b.n_blocks, b.sblk0.p, b.n_star_blocks, b.big_stars.p, b.n_big_stars,
                 static_cast<int32_t>(b.g.size()), in, C, s);
    run_chain(batch_view(b, spec), spec, in, out, C, lanes, ct, s);
}

void config_for(const Batch& b, int32_t C, int& lanes, int& ct) {
    lanes = b.lanes[C] ? b.lanes[C] : (g_hop_lanes == AHR_HOP_AUTO ? 4 : g_hop_lanes);
    ct = b.ct[C] ? b.ct[C] : C;
}

void batch_filter(Batch& b, const ahr_filter_spec& spec, const float* in, float* out, int32_t C, bool use_graph,
                  int lanes, int ct, hipStream_t s) {
    ensure_operator(b, spec, s);
    float alpha_sum = 0.f;
    if (spec_kmax(spec, &alpha_sum) == 0) {
        const int64_t n = static_cast<int64_t>(b.n_inst) * C;
        hipLaunchKernelGGL(k_batch_identity, dim3(grid_for(n, kBT)), dim3(kBT), 0, s, n, C, b.flags.p, in, out,
                           alpha_sum);
        AHR_LAUNCHED("k_batch_identity");
        return;
    }
    if (lanes == AHR_HOP_ROW_BLOCK) row_blocks(b.net_rp.p, b.hint_rp.p, b.n_tot, b.n_inst, b.rc, b.scan_tmp, s);
    const size_t nz = static_cast<size_t>(b.n_tot) * C;
    b.z0.ensure(nz, s);
    b.z1.ensure(nz, s);
    b.acc.ensure(nz, s);
    if (!use_graph) {
        // the descriptors' host copy must outlive the copy: wait for it
        AHR_HIP(hipStreamSynchronize(s));
        b.eager_host = descriptors(b, spec, C, ct);
        b.eager_desc.ensure(b.eager_host.size(), s);
        AHR_HIP(hipMemcpyAsync(b.eager_desc.p, b.eager_host.data(), b.eager_host.size() * sizeof(ExpandArgs),
                               hipMemcpyHostToDevice, s));
        enqueue(b, b.eager_desc.p, spec, in, out, C, lanes, ct, s);
        return;
    }
    Captured* hit = nullptr;
    for (Captured* c : b.cache)
        if (c->C == C && c->lanes == lanes && c->ct == ct && c->in == in && c->out == out && c->z0 == b.z0.p &&
            same_spec(c->spec, spec)) {
            hit = c;
            break;
        }
    if (!hit) {
        if (b.cache.size() >= kCacheMax) {
            auto it = std::min_element(b.cache.begin(), b.cache.end(),
                                       [](const Captured* x, const Captured* y) { return x->used < y->used; });
            AHR_HIP(hipStreamSynchronize(s));
            drop(*it, s);
            b.cache.erase(it);
        }
        auto* c = new Captured();
        c->spec = spec;
        c->C = C;
        c->lanes = lanes;
        c->ct = ct;
        c->in = in;
        c->out = out;
        c->z0 = b.z0.p;
        try {
            c->host_desc = descriptors(b, spec, C, ct);
            c->desc.ensure(c->host_desc.size(), s);
            AHR_HIP(hipMemcpyAsync(c->desc.p, c->host_desc.data(), c->host_desc.size() * sizeof(ExpandArgs),
                                   hipMemcpyHostToDevice, s));
            AHR_HIP(hipStreamSynchronize(s));
            if (!b.cap_stream) AHR_HIP(hipStreamCreateWithFlags(&b.cap_stream, hipStreamNonBlocking));
            const hipStream_t cs = b.cap_stream;
            hipGraph_t graph = nullptr;
            AHR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            set_capture(true);
            try {
                enqueue(b, c->desc.p, spec, in, out, C, lanes, ct, cs);
            } catch (...) {
                set_capture(false);
                hipGraph_t broken = nullptr;
                (void)hipStreamEndCapture(cs, &broken);
                if (broken) (void)hipGraphDestroy(broken);
                throw;
            }
            set_capture(false);
            AHR_HIP(hipStreamEndCapture(cs, &graph));
            hipError_t e = hipGraphInstantiate(&c->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            AHR_HIP(e);
        } catch (...) {
            drop(c, s);
            throw;
        }
        b.cache.push_back(c);
        hit = c;
    }
    hit->used = ++b.clock;
    AHR_HIP(hipGraphLaunch(hit->exec, s));
}

}  // namespace

Batch::~Batch() {
    hipStream_t s = nullptr;
    (void)hipDeviceSynchronize();
    for (Captured* c : cache) drop(c, s);
    for (Graph* x : g) delete x;
    net_rp.release(s);
    hint_rp.release(s);
    net_ent.release(s);
    hint_ent.release(s);
    perm.release(s);
    flags.release(s);
    scale.release(s);
    coef.release(s);
    rc.release(s);
    blk0.release(s);
    sblk0.release(s);
    big_stars.release(s);
    z0.release(s);
    z1.release(s);
    acc.release(s);
    scan_tmp.release(s);
    eager_desc.release(s);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

// Concatenate the member graphs' rows (netlist and hint lists) into the
// batch rows, with columns mapped to batch rows.
void batch_rows(Batch& b, bool hints, DevBuf<int32_t>& rp, DevBuf<int2>& ent, int64_t& nnz, hipStream_t s) {
    DevBuf<int32_t> len;
    len.ensure(static_cast<size_t>(b.n_tot) + 1, s);
    for (size_t i = 0; i < b.g.size(); ++i) {
        Graph& g = *b.g[i];
        const int32_t* grp = hints ? g.xhint_rp.p : g.xnet_rp.p;
        hipLaunchKernelGGL(k_batch_row_lens, dim3(grid_for(g.n_tot, kBT)), dim3(kBT), 0, s, g.n_tot, g.n_inst,
                           b.inst0[i], b.aux0[i], grp, len.p);
        AHR_LAUNCHED("k_batch_row_lens");
    }
    rp.ensure(static_cast<size_t>(b.n_tot) + 1, s);
    b.scan_tmp.ensure(scan_tmp_elems(b.n_tot), s);
    nnz = scan_i32_checked(len.p, rp.p, b.n_tot, b.scan_tmp.p, s);
    len.release(s);
    if (nnz >= (int64_t(1) << 31)) throw Error{AHR_EUNSUPPORTED, "batch has 2^31 or more entries in one list"};
    ent.ensure(static_cast<size_t>(nnz) + 1, s);
    for (size_t i = 0; i < b.g.size(); ++i) {
        Graph& g = *b.g[i];
        const int32_t* grp = hints ? g.xhint_rp.p : g.xnet_rp.p;
        const int2* gent = hints ? g.xhint_ent.p : net_entries(g, s);
        hipLaunchKernelGGL(k_batch_copy_rows, dim3(grid_for(static_cast<int64_t>(g.n_tot) * kWave, kBT)), dim3(kBT), 0,
                           s, g.n_tot, g.n_inst, b.inst0[i], b.aux0[i], grp, gent, rp.p, ent.p);
        AHR_LAUNCHED("k_batch_copy_rows");
    }
}

void batch_assemble(Batch& b, hipStream_t s) {
    const size_t n = b.g.size();
    b.inst0.assign(n, 0);
    b.aux0.assign(n, 0);
    int64_t ni = 0, na = 0;
    for (size_t i = 0; i < n; ++i) ni += b.g[i]->n_inst;
    for (size_t i = 0; i < n; ++i) {
        na += b.g[i]->n_tot - b.g[i]->n_inst;
    }
    if (ni + na >= (int64_t(1) << 31)) throw Error{AHR_EUNSUPPORTED, "batch has 2^31 or more rows"};
    int64_t oi = 0, oa = ni;
    for (size_t i = 0; i < n; ++i) {
        b.inst0[i] = static_cast<int32_t>(oi);
        b.aux0[i] = static_cast<int32_t>(oa);
        oi += b.g[i]->n_inst;
        oa += b.g[i]->n_tot - b.g[i]->n_inst;
    }
    b.n_inst = static_cast<int32_t>(ni);
    b.n_tot = static_cast<int32_t>(ni + na);
    batch_rows(b, false, b.net_rp, b.net_ent, b.nnz_net, s);
    batch_rows(b, true, b.hint_rp, b.hint_ent, b.nnz_hint, s);
    b.perm.ensure(static_cast<size_t>(b.n_inst) + 1, s);
    b.flags.ensure(static_cast<size_t>(b.n_inst) + 1, s);
    for (size_t i = 0; i < n; ++i) {
        Graph& g = *b.g[i];
        hipLaunchKernelGGL(k_batch_inst, dim3(grid_for(g.n_inst, kBT)), dim3(kBT), 0, s, g.n_inst, b.inst0[i], g.perm.p,
                           g.nl.node_flags, b.perm.p, b.flags.p);
        AHR_LAUNCHED("k_batch_inst");
    }
    b.scale.ensure(static_cast<size_t>(b.n_tot) + 1, s);
    b.coef.ensure(static_cast<size_t>(b.n_tot) + 1, s);
    b.op_version.assign(n, -1);
    row_classes(b.net_rp.p, b.hint_rp.p, b.n_tot, b.n_inst, b.rc, b.scan_tmp, s);
    std::vector<int32_t> blk(n + 1, 0), sblk(n + 1, 0);
    for (size_t i = 0; i < n; ++i) {
        blk[i + 1] = blk[i] + static_cast<int32_t>(grid_for(b.g[i]->n_tot, kBT));
        sblk[i + 1] = sblk[i] + b.g[i]->n_star;
    }
    b.n_blocks = blk[n];
    b.n_star_blocks = sblk[n];
    b.blk0.ensure(n + 1, s);
    b.sblk0.ensure(n + 1, s);
    AHR_HIP(hipMemcpyAsync(b.blk0.p, blk.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    AHR_HIP(hipMemcpyAsync(b.sblk0.p, sblk.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    // big stars of every member, as batch star indices
    std::vector<int32_t> big;
    for (size_t i = 0; i < n; ++i) {
        Graph& g = *b.g[i];
        if (!g.n_big_stars) continue;
        std::vector<int32_t> loc(g.n_big_stars);
        AHR_HIP(hipMemcpyAsync(loc.data(), g.big_stars.p, loc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        AHR_HIP(hipStreamSynchronize(s));
        for (int32_t k : loc) big.push_back(sblk[i] + k);
    }
    b.n_big_stars = static_cast<int32_t>(big.size());
    b.big_stars.ensure(big.size() + 1, s);
    if (!big.empty())
        AHR_HIP(hipMemcpyAsync(b.big_stars.p, big.data(), big.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    AHR_HIP(hipStreamSynchronize(s));
}

}  // namespace ahr

using ahr::Batch;
using ahr::fail;

namespace {

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }
bool ncols_ok(int32_t c) { return c == 1 || c == 2 || c == 4 || c == 8; }
bool pow2_lanes(int32_t l) { return l == AHR_HOP_ROW_BLOCK || (l >= 1 && l <= 64 && (l & (l - 1)) == 0); }
bool tile_ok(int32_t C, int32_t ct) { return ct >= 1 && ct <= C && C % ct == 0 && (ct & (ct - 1)) == 0; }

template <class F>
ahr_status guarded_b(F&& f) {
    struct Flush {
        ~Flush() { ahr::flush_frees(); }
    } flush;
    try {
        ahr::set_error(AHR_OK, "");
        return f();
    } catch (const ahr::Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(AHR_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(AHR_EDEVICE, "unexpected exception");
    }
}

}  // namespace

extern "C" {

ahr_status ahr_batch_build(const ahr_netlist* nls, const ahr_hint_params* hps, int32_t n, const float* pos,
                           int32_t ncols, void* stream, ahr_batch** out) {
    if (!out) return fail(AHR_EINVAL, "out is NULL");
    if (!nls || !hps || !pos) return fail(AHR_EINVAL, "netlists, hint params and placement are required");
    if (n < 1 || n > 65536) return fail(AHR_EINVAL, "n in [1, 65536]");
    if (!ncols_ok(ncols) || ncols < 2) return fail(AHR_EINVAL, "ncols must be 2, 4 or 8");
    for (int32_t i = 0; i < n; ++i) {
        const ahr_netlist& nl = nls[i];
        if (nl.n_inst <= 0 || nl.n_nets < 0 || nl.n_pins < 0 || !nl.net_ptr || !nl.node_flags || !nl.node_size ||
            (nl.n_pins > 0 && (!nl.pin_node || !nl.pin_off)) || nl.reserved0 != 0)
            return fail(AHR_EINVAL, "netlist " + std::to_string(i) + " is invalid");
        if (!(nl.die[0] < nl.die[2]) || !(nl.die[1] < nl.die[3])) return fail(AHR_EINVAL, "empty die");
        const ahr_hint_params& hp = hps[i];
        if (hp.nbx < 1 || hp.nby < 1 || hp.nbx > 4096 || hp.nby > 4096 ||
            static_cast<int64_t>(hp.nbx) * hp.nby > 16384 || !(hp.mu > 0.f) || hp.clique_max < 1 ||
            !(hp.detection_ratio >= 0.f && hp.detection_ratio <= 1.f) || (hp.flags & ~AHR_ALL_HINTS))
            return fail(AHR_EINVAL, "hint params " + std::to_string(i) + " are invalid");
    }
    return guarded_b([&]() -> ahr_status {
        hipStream_t s = as_stream(stream);
        auto* b = new Batch();
        try {
            AHR_HIP(hipGetDevice(&b->device));
            int64_t off = 0;
            for (int32_t i = 0; i < n; ++i) {
                auto* g = new ahr::Graph();
                b->g.push_back(g);
                g->nl = nls[i];
                g->hp = hps[i];
                g->device = b->device;
                ahr::build_netlist(*g, s);
                ahr::build_hints(*g, pos + off * ncols, ncols, s);
                off += nls[i].n_inst;
            }
            ahr::batch_assemble(*b, s);
        } catch (...) {
            delete b;
            throw;
        }
        *out = reinterpret_cast<ahr_batch*>(b);
        return AHR_OK;
    });
}

ahr_status ahr_batch_get_info(const ahr_batch* h, ahr_batch_info* info) {
    if (!h || !info) return fail(AHR_EINVAL, "NULL argument");
    const auto* b = reinterpret_cast<const Batch*>(h);
    std::memset(info, 0, sizeof *info);
    info->n_graphs = static_cast<int32_t>(b->g.size());
    info->n_inst = b->n_inst;
    info->n_tot = b->n_tot;
    info->nnz_net = b->nnz_net;
    info->nnz_hint = b->nnz_hint;
    info->n_long_rows = b->rc.n_long;
    info->n_captured = static_cast<int32_t>(b->cache.size());
    return AHR_OK;
}

ahr_status ahr_batch_set_config(ahr_batch* h, int32_t ncols, int32_t lanes_per_row, int32_t col_tile) {
    if (!h) return fail(AHR_EINVAL, "batch is NULL");
    if (!ncols_ok(ncols)) return fail(AHR_EINVAL, "ncols must be 1, 2, 4 or 8");
    if (lanes_per_row != 0 && !pow2_lanes(lanes_per_row))
        return fail(AHR_EINVAL,
                    "lanes_per_row must be a power of two in [1, 64], AHR_HOP_ROW_BLOCK, or 0 for the default");
    if (col_tile != 0 && !tile_ok(ncols, col_tile))
        return fail(AHR_EINVAL, "col_tile must be a power of two dividing ncols, or 0 for ncols");
    auto* b = reinterpret_cast<Batch*>(h);
    b->lanes[ncols] = lanes_per_row;
    b->ct[ncols] = col_tile;
    return AHR_OK;
}

ahr_status ahr_batch_get_config(const ahr_batch* h, int32_t ncols, int32_t* lanes_per_row, int32_t* col_tile) {
    if (!h || !lanes_per_row || !col_tile) return fail(AHR_EINVAL, "NULL argument");
    if (!ncols_ok(ncols)) return fail(AHR_EINVAL, "ncols must be 1, 2, 4 or 8");
    int lanes, ct;
    ahr::config_for(*reinterpret_cast<const Batch*>(h), ncols, lanes, ct);
    *lanes_per_row = lanes;
    *col_tile = ct;
    return AHR_OK;
}

ahr_status ahr_batch_filter(ahr_batch* h, const ahr_filter_spec* spec, const float* in, float* out, int32_t ncols,
                            int32_t use_graph, void* stream) {
    if (!h) return fail(AHR_EINVAL, "batch is NULL");
    if (!spec) return fail(AHR_EINVAL, "filter spec is NULL");
    if (spec->nbands < 1 || spec->nbands > AHR_MAX_BANDS) return fail(AHR_EINVAL, "nbands in [1, 4]");
    for (int i = 0; i < spec->nbands; ++i)
        if (spec->k[i] < 0 || spec->k[i] > 64 || !std::isfinite(spec->alpha[i]))
            return fail(AHR_EINVAL, "k in [0, 64], finite alpha");
    if (!(spec->sigma >= 0.f) || !std::isfinite(spec->sigma)) return fail(AHR_EINVAL, "sigma must be >= 0");
    if (spec->lambda_mode != AHR_LAMBDA_GERSHGORIN && spec->lambda_mode != AHR_LAMBDA_FIXED)
        return fail(AHR_EINVAL, "unknown lambda_mode");
    if (spec->lambda_mode == AHR_LAMBDA_FIXED && !(spec->lambda_fixed >= 0.f && std::isfinite(spec->lambda_fixed)))
        return fail(AHR_EINVAL, "lambda_fixed must be >= 0");
    if (!in || !out) return fail(AHR_EINVAL, "in/out is NULL");
    if (!ncols_ok(ncols)) return fail(AHR_EINVAL, "ncols must be 1, 2, 4 or 8");
    auto* b = reinterpret_cast<Batch*>(h);
    const size_t bytes = static_cast<size_t>(b->n_inst) * ncols * sizeof(float);
    auto x = reinterpret_cast<uintptr_t>(in), y = reinterpret_cast<uintptr_t>(out);
    if (x < y + bytes && y < x + bytes) return fail(AHR_EINVAL, "in and out overlap");
    return guarded_b([&]() -> ahr_status {
        int lanes, ct;
        ahr::config_for(*b, ncols, lanes, ct);
        ahr::batch_filter(*b, *spec, in, out, ncols, use_graph != 0, lanes, ct, as_stream(stream));
        return AHR_OK;
    });
}

ahr_status ahr_batch_autotune(ahr_batch* h, const ahr_filter_spec* spec, int32_t ncols, void* stream,
                              int32_t* lanes_per_row, int32_t* col_tile, float* best_ms) {
    if (!h || !spec) return fail(AHR_EINVAL, "NULL argument");
    if (!ncols_ok(ncols)) return fail(AHR_EINVAL, "ncols must be 1, 2, 4 or 8");
    auto* b = reinterpret_cast<Batch*>(h);
    return guarded_b([&]() -> ahr_status {
        hipStream_t s = as_stream(stream);
        const int64_t n = static_cast<int64_t>(b->n_inst) * ncols;
        ahr::DevBuf<float> in, out;
        in.ensure(static_cast<size_t>(n), s);
        out.ensure(static_cast<size_t>(n), s);
        hipLaunchKernelGGL(ahr::k_batch_pattern, dim3(ahr::grid_for(n, 256)), dim3(256), 0, s, n, in.p);
        AHR_LAUNCHED("k_batch_pattern");
        hipEvent_t e0, e1;
        AHR_HIP(hipEventCreate(&e0));
        AHR_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        int best_l = 0, best_t = 0;
        std::vector<ahr::Captured*> before = b->cache;
        try {
            const int cand[] = {1, 2, 4, 8, 16, 32, AHR_HOP_ROW_BLOCK};
            for (int lanes : cand)
                for (int ct = ncols; ct >= 1; ct >>= 1) {
                    ahr::batch_filter(*b, *spec, in.p, out.p, ncols, true, lanes, ct, s);   // capture + warm
                    ahr::batch_filter(*b, *spec, in.p, out.p, ncols, true, lanes, ct, s);
                    constexpr int kReps = 3;
                    AHR_HIP(hipEventRecord(e0, s));
                    for (int r = 0; r < kReps; ++r) ahr::batch_filter(*b, *spec, in.p, out.p, ncols, true, lanes, ct, s);
                    AHR_HIP(hipEventRecord(e1, s));
                    AHR_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    AHR_HIP(hipEventElapsedTime(&ms, e0, e1));
                    ms /= kReps;
                    if (ms < best) {
                        best = ms;
                        best_l = lanes;
                        best_t = ct;
                    }
                    // drop this candidate's capture (its buffers are the tuner's own)
                    for (auto it = b->cache.begin(); it != b->cache.end();) {
                        if ((*it)->in == in.p && std::find(before.begin(), before.end(), *it) == before.end()) {
                            ahr::drop(*it, s);
                            it = b->cache.erase(it);
                        } else {
                            ++it;
                        }
                    }
                }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            in.release(s);
            out.release(s);
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        in.release(s);
        out.release(s);
        b->lanes[ncols] = best_l;
        b->ct[ncols] = best_t;
        if (lanes_per_row) *lanes_per_row = best_l;
        if (col_tile) *col_tile = best_t;
        if (best_ms) *best_ms = best;
        return AHR_OK;
    });
}

void ahr_batch_destroy(ahr_batch* h) {
    if (!h) return;
    try {
        delete reinterpret_cast<Batch*>(h);
    } catch (...) {
    }
    ahr::flush_frees();
}

}  // extern "C"
