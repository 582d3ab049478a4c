// C entry points: argument validation, error capture, orchestration.
#include <cmath>
#include <cstring>

#include "ahr_internal.hpp"

namespace ahr {

std::string& last_error_ref();
extern int g_hop_lanes;
extern int g_hop_nt;

int32_t net_count(const Graph& g, hipStream_t s) {
    if (g.nnz_net >= 0) return g.nnz_net;
    if (g.has_layout) {
        g.nnz_net = read_i32(g.xnet_rp.p + g.n_tot, s);
    } else {       // before any placement: add up the merged row lengths
        DevBuf<int32_t> pre;
        DevBuf<int64_t> tmp;
        pre.ensure(static_cast<size_t>(g.n_tot) + 1, s);
        tmp.ensure(scan_tmp_elems(g.n_tot), s);
        g.nnz_net = static_cast<int32_t>(scan_i32_checked(g.net_len.p, pre.p, g.n_tot, tmp.p, s));
        pre.release(s);
        tmp.release(s);
    }
    return g.nnz_net;
}

int32_t hint_count(const Graph& g, hipStream_t s) {
    if (g.nnz_hint < 0) g.nnz_hint = read_i32(g.xhint_rp.p + g.n_tot, s);
    return g.nnz_hint;
}

Graph::~Graph() {
    // one stream: its later work (and any other stream, through the block
    // events) reuses the memory only after this graph's work.  Several
    // streams: wait for the whole device first (a null-stream wait would not
    // cover non-blocking streams), then release.
    hipStream_t s = stream_uses == 1 ? work_stream : nullptr;
    if (stream_uses > 1) (void)hipDeviceSynchronize();
    if (xnet_ready) (void)hipStreamWaitEvent(s, xnet_ready, 0);   // the side stream's copy
    DevBuf<int32_t>* i32[] = {&pin_node_x, &mpin_owner, &mpin_pin, &star_net, &macro_ids, &net_len, &net_col,
                              &big_nets, &cell_bin, &bin_start, &bin_cells, &bm_start, &bm_list, &hint_cnt,
                              &nmac, &nwin, &bin_rank, &wpre, &pair_off, &pair_row, &pair_mac, &mlist, &mstart,
                              &big_stars, &i32a, &i32b, &counter, &kept, &loc_flag};
    for (auto* b : i32) b->release(s);
    loc_part.release(s);
    keep_mask.release(s);
    net_q.release(s);
    net_off.release(s);
    perm.release(s);
    iperm.release(s);
    xmpin.release(s);
    xstar_net.release(s);
    xnet_rp.release(s);
    xnet_ent.release(s);
    xqdeg.release(s);
    xhint_rp.release(s);
    xhint_ent.release(s);
    lay_start.release(s);
    qdeg.release(s);
    base_w.release(s);
    xcell.release(s);
    xbase_w.release(s);
    xpos.release(s);
    xhabs.release(s);
    xhsg.release(s);
    gmax.release(s);
    bin_area_q.release(s);
    macro_area_q.release(s);
    phi.release(s);
    macro_span.release(s);
    macro_rect.release(s);
    deg.release(s);
    scale.release(s);
    hsum.release(s);
    for (auto& z : zh) z.release(s);
    lam.release(s);
    coef.release(s);
    rc.release(s);
    z0.release(s);
    zpk.release(s);
    z1.release(s);
    acc.release(s);
    ga.release(s);
    gb.release(s);
    gt.release(s);
    scan_tmp.release(s);
    i64a.release(s);
    arena_destroy(arena);
    if (xnet_fork) (void)hipEventDestroy(xnet_fork);
    if (xnet_ready) (void)hipEventDestroy(xnet_ready);
}

}  // namespace ahr

using ahr::Error;
using ahr::fail;

namespace {

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

bool ncols_ok(int32_t c) { return c == 1 || c == 2 || c == 4 || c == 8; }

ahr_status check_netlist(const ahr_netlist* nl) {
    if (!nl) return fail(AHR_EINVAL, "netlist is NULL");
    if (nl->n_inst <= 0) return fail(AHR_EINVAL, "n_inst must be positive");
    if (nl->n_nets < 0 || nl->n_pins < 0) return fail(AHR_EINVAL, "negative net or pin count");
    if (nl->reserved0 != 0) return fail(AHR_EINVAL, "reserved0 must be 0");
    if (!nl->net_ptr || !nl->node_flags || !nl->node_size)
        return fail(AHR_EINVAL, "net_ptr, node_flags and node_size are required");
    if (nl->n_pins > 0 && (!nl->pin_node || !nl->pin_off)) return fail(AHR_EINVAL, "pin_node/pin_off is NULL");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(nl->die[k])) return fail(AHR_EINVAL, "die is not finite");
    if (!(nl->die[0] < nl->die[2]) || !(nl->die[1] < nl->die[3])) return fail(AHR_EINVAL, "empty die");
    return AHR_OK;
}

ahr_status check_hints(const ahr_hint_params* hp) {
    if (!hp) return fail(AHR_EINVAL, "hint params are NULL");
    if (hp->nbx < 1 || hp->nby < 1 || hp->nbx > 4096 || hp->nby > 4096) return fail(AHR_EINVAL, "nbx, nby in [1, 4096]");
    if (static_cast<int64_t>(hp->nbx) * hp->nby > 16384)
        return fail(AHR_EUNSUPPORTED, "at most 16384 bins (nbx * nby)");
    if (!(hp->detection_ratio >= 0.f && hp->detection_ratio <= 1.f)) return fail(AHR_EINVAL, "detection_ratio in [0, 1]");
    if (!(hp->mu > 0.f) || !std::isfinite(hp->mu)) return fail(AHR_EINVAL, "mu must be positive");
    if (!std::isfinite(hp->bin_capacity)) return fail(AHR_EINVAL, "bin_capacity must be finite");
    if (hp->clique_max < 1) return fail(AHR_EINVAL, "clique_max must be >= 1");
    if (hp->flags & ~(AHR_ALL_HINTS | AHR_LAYOUT_AUTO | AHR_LAYOUT_NETLIST))
        return fail(AHR_EINVAL, "unknown hint flags");
    if ((hp->flags & AHR_LAYOUT_AUTO) && (hp->flags & AHR_LAYOUT_NETLIST))
        return fail(AHR_EINVAL, "AHR_LAYOUT_AUTO and AHR_LAYOUT_NETLIST exclude each other");
    if (!(hp->prune_tau >= 0.f && hp->prune_tau <= 1.f)) return fail(AHR_EINVAL, "prune_tau in [0, 1]");
    return AHR_OK;
}

ahr_status check_spec(const ahr_filter_spec* sp) {
    if (!sp) return fail(AHR_EINVAL, "filter spec is NULL");
    if (sp->nbands < 1 || sp->nbands > AHR_MAX_BANDS) return fail(AHR_EINVAL, "nbands in [1, 4]");
    for (int b = 0; b < sp->nbands; ++b) {
        if (sp->k[b] < 0 || sp->k[b] > 64) return fail(AHR_EINVAL, "k in [0, 64]");
        if (!std::isfinite(sp->alpha[b])) return fail(AHR_EINVAL, "alpha must be finite");
    }
    if (!(sp->sigma >= 0.f) || !std::isfinite(sp->sigma)) return fail(AHR_EINVAL, "sigma must be >= 0");
    if (sp->lambda_mode != AHR_LAMBDA_GERSHGORIN && sp->lambda_mode != AHR_LAMBDA_FIXED)
        return fail(AHR_EINVAL, "unknown lambda_mode");
    if (sp->lambda_mode == AHR_LAMBDA_FIXED && !(sp->lambda_fixed >= 0.f && std::isfinite(sp->lambda_fixed)))
        return fail(AHR_EINVAL, "lambda_fixed must be >= 0");
    return AHR_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

template <class F>
ahr_status guarded(F&& f) {
    struct Flush {
        ~Flush() { ahr::flush_frees(); }
    } flush;
    try {
        ahr::set_error(AHR_OK, "");
        return f();
    } catch (const Error& e) {
        return fail(e.code, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(AHR_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(AHR_EDEVICE, "unexpected exception");
    }
}

}  // namespace

extern "C" {

const char* ahr_version(void) { return "ahr 0.1 gfx950"; }

const char* ahr_last_error(void) { return ahr::last_error_ref().c_str(); }

ahr_status ahr_graph_workspace_size(const ahr_netlist* nl, const ahr_hint_params* hp, int32_t ncols, void* stream,
                                    size_t* bytes) {
    ahr_status st;
    if ((st = check_netlist(nl)) != AHR_OK) return st;
    if ((st = check_hints(hp)) != AHR_OK) return st;
    if (!bytes) return fail(AHR_EINVAL, "bytes is NULL");
    if (!ncols_ok(ncols)) return fail(AHR_EINVAL, "ncols must be 1, 2, 4 or 8");
    return guarded([&]() -> ahr_status {
        *bytes = ahr::graph_workspace_bytes(*nl, *hp, ncols, as_stream(stream));
        return AHR_OK;
    });
}

namespace {

// Build a graph (in the workspace when one is given): the body of
// ahr_graph_build and of the netlist form of ahr_refine.
// bound_cols: the most columns later calls will use (the workspace bound).
ahr::Graph* new_graph(const ahr_netlist* nl, const ahr_hint_params* hp, const float* g, int32_t ncols,
                      int32_t bound_cols, void* ws, size_t ws_bytes, hipStream_t s) {
    ahr::Arena* arena = nullptr;
    if (ws) {
        arena = ahr::arena_create(ws, ws_bytes);
        try {
            ahr::ArenaScope scope(arena);
            const size_t need = ahr::graph_workspace_bytes(*nl, *hp, bound_cols, s);
            if (ws_bytes < need) {
                char buf[160];
                snprintf(buf, sizeof buf, "workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
                throw Error{AHR_ENOMEM, buf};
            }
        } catch (...) {
            ahr::arena_destroy(arena);
            throw;
        }
    }
    auto* gr = new ahr::Graph();
    gr->arena = arena;
    ahr::ArenaScope scope(arena);
    gr->use_stream(s);
    gr->nl = *nl;
    gr->hp = *hp;
    try {
        AHR_HIP(hipGetDevice(&gr->device));
        ahr::build_netlist(*gr, s);
        if (g) ahr::build_hints(*gr, g, ncols, s);
    } catch (...) {
        delete gr;
        throw;
    }
    return gr;
}

}  // namespace

ahr_status ahr_graph_build(const ahr_netlist* nl, const ahr_hint_params* hp, const float* g, int32_t ncols, void* ws,
                           size_t ws_bytes, void* stream, ahr_graph** out) {
    ahr_status st;
    if ((st = check_netlist(nl)) != AHR_OK) return st;
    if ((st = check_hints(hp)) != AHR_OK) return st;
    if (!out) return fail(AHR_EINVAL, "out is NULL");
    if (g && (!ncols_ok(ncols) || ncols < 2)) return fail(AHR_EINVAL, "ncols must be 2, 4 or 8 with a placement");
    if (ws && ws_bytes < ahr::graph_workspace_floor(*nl, g ? ncols : 8))
        return fail(AHR_ENOMEM, "workspace too small for the netlist's sizes (ask ahr_graph_workspace_size)");
    return guarded([&]() -> ahr_status {
        hipStream_t s = as_stream(stream);
        auto* gr = new_graph(nl, hp, g, ncols, g ? ncols : 8, ws, ws_bytes, s);
        if (g) {
            try {
                AHR_HIP(hipStreamSynchronize(s));
            } catch (...) {
                delete gr;
                throw;
            }
        }
        *out = reinterpret_cast<ahr_graph*>(gr);
        return AHR_OK;
    });
}

ahr_status ahr_graph_update_hints(ahr_graph* h, const float* g, int32_t ncols, void* stream) {
    if (!h) return fail(AHR_EINVAL, "graph is NULL");
    if (!g) return fail(AHR_EINVAL, "placement is NULL");
    if (!ncols_ok(ncols) || ncols < 2) return fail(AHR_EINVAL, "ncols must be 2, 4 or 8");
    return guarded([&]() -> ahr_status {
        ahr::ArenaScope arena_scope(reinterpret_cast<const ahr::Graph*>(h)->arena);
        auto* gr = reinterpret_cast<ahr::Graph*>(h);
        hipStream_t s = as_stream(stream);
        gr->use_stream(s);
        ahr::build_hints(*gr, g, ncols, s);
        AHR_HIP(hipStreamSynchronize(s));
        return AHR_OK;
    });
}

ahr_status ahr_graph_get_info(const ahr_graph* h, ahr_graph_info* info) {
    if (!h || !info) return fail(AHR_EINVAL, "NULL argument");
    return guarded([&]() -> ahr_status {
        ahr::ArenaScope arena_scope(reinterpret_cast<const ahr::Graph*>(h)->arena);
        const auto* g = reinterpret_cast<const ahr::Graph*>(h);
        // entry counts not read yet come from the row pointers, on the
        // stream the graph's work went to (after a device wait when it went
        // to several: the null stream does not wait for non-blocking ones)
        const hipStream_t s = g->stream_uses == 1 ? g->work_stream : nullptr;
        if (g->stream_uses > 1 && (g->nnz_net < 0 || (g->has_hints && g->nnz_hint < 0)))
            AHR_HIP(hipDeviceSynchronize());
        const int32_t nnz_net = ahr::net_count(*g, s);
        const int32_t nnz_hint = g->has_hints ? ahr::hint_count(*g, s) : 0;
        std::memset(info, 0, sizeof *info);
        info->n_inst = g->n_inst;
        info->n_tot = g->n_tot;
        info->first_mpin = g->first_mpin;
        info->first_star = g->first_star;
        info->first_mvirt = g->first_mvirt;
        info->first_bvirt = g->first_bvirt;
        info->nnz_net = nnz_net;
        info->nnz_hint = nnz_hint;
        info->n_hint_cells = g->n_hint_cells;
        info->n_long_rows = g->rc.n_long;
        info->hint_version = g->hint_version;
        info->layout = g->layout_netlist;
        info->hop_lanes = g->hop_local < 0 ? 0 : (g->hop_local ? 4 : AHR_HOP_ROW_BLOCK);
        info->reserved = 0;
        info->ws_bytes = static_cast<int64_t>(ahr::arena_size(g->arena));
        info->ws_peak = static_cast<int64_t>(ahr::arena_peak(g->arena));
        return AHR_OK;
    });
}

ahr_status ahr_graph_export(const ahr_graph* h, ahr_graph_host* dst, void* stream) {
    if (!h || !dst) return fail(AHR_EINVAL, "NULL argument");
    return guarded([&]() -> ahr_status {
        ahr::ArenaScope arena_scope(reinterpret_cast<const ahr::Graph*>(h)->arena);
        const auto* g = reinterpret_cast<const ahr::Graph*>(h);
        hipStream_t s = as_stream(stream);
        g->use_stream(s);
        const size_t N = static_cast<size_t>(g->n_tot);
        auto cp = [&](void* d, const void* src, size_t bytes) {
            if (d && bytes) AHR_HIP(hipMemcpyAsync(d, src, bytes, hipMemcpyDeviceToHost, s));
        };
        if (dst->net_row_ptr || dst->net_col || dst->net_q) {
            // the merged rows sit in place on the device: pack them
            std::vector<int64_t> off(N + 1);
            std::vector<int32_t> len(N + 1);
            AHR_HIP(hipMemcpyAsync(off.data(), g->net_off.p, (N + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
            AHR_HIP(hipMemcpyAsync(len.data(), g->net_len.p, N * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            AHR_HIP(hipStreamSynchronize(s));
            std::vector<int32_t> rp(N + 1, 0);
            for (size_t r = 0; r < N; ++r) rp[r + 1] = rp[r] + len[r];
            if (dst->net_row_ptr) std::memcpy(dst->net_row_ptr, rp.data(), (N + 1) * sizeof(int32_t));
            const size_t cap = static_cast<size_t>(off[N]);
            if (dst->net_col && cap) {
                std::vector<int32_t> col(cap);
                AHR_HIP(hipMemcpyAsync(col.data(), g->net_col.p, cap * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                AHR_HIP(hipStreamSynchronize(s));
                for (size_t r = 0; r < N; ++r)
                    std::memcpy(dst->net_col + rp[r], col.data() + off[r], static_cast<size_t>(len[r]) * sizeof(int32_t));
            }
            if (dst->net_q && cap) {
                std::vector<int64_t> q(cap);
                AHR_HIP(hipMemcpyAsync(q.data(), g->net_q.p, cap * sizeof(int64_t), hipMemcpyDeviceToHost, s));
                AHR_HIP(hipStreamSynchronize(s));
                for (size_t r = 0; r < N; ++r)
                    std::memcpy(dst->net_q + rp[r], q.data() + off[r], static_cast<size_t>(len[r]) * sizeof(int64_t));
            }
        }
        if (g->has_hints && (dst->hint_row_ptr || dst->hint_col || dst->hint_val)) {
            // hint rows live in execution order: return them in node order
            const size_t np = static_cast<size_t>(g->first_mvirt);     // rows the layout permutes
            std::vector<int32_t> xrp(N + 1), perm(np);
            const int32_t nnz_hint = ahr::hint_count(*g, s);
            std::vector<int2> ent(nnz_hint);
            AHR_HIP(hipMemcpyAsync(xrp.data(), g->xhint_rp.p, (N + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            AHR_HIP(hipMemcpyAsync(perm.data(), g->perm.p, np * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            if (nnz_hint)
                AHR_HIP(hipMemcpyAsync(ent.data(), g->xhint_ent.p, nnz_hint * sizeof(int2), hipMemcpyDeviceToHost, s));
            AHR_HIP(hipStreamSynchronize(s));
            std::vector<int32_t> iperm(np);
            for (size_t r = 0; r < np; ++r) iperm[perm[r]] = static_cast<int32_t>(r);
            std::vector<int32_t> rp(N + 1, 0);
            for (size_t c = 0; c < N; ++c) {
                size_t r = c < np ? static_cast<size_t>(iperm[c]) : c;
                rp[c + 1] = rp[c] + (xrp[r + 1] - xrp[r]);
            }
            if (dst->hint_row_ptr) std::memcpy(dst->hint_row_ptr, rp.data(), (N + 1) * sizeof(int32_t));
            for (size_t c = 0; c < N; ++c) {
                size_t r = c < np ? static_cast<size_t>(iperm[c]) : c;
                for (int32_t k = xrp[r]; k < xrp[r + 1]; ++k) {
                    int32_t o = rp[c] + (k - xrp[r]);
                    int32_t col = ent[k].x;
                    if (dst->hint_col) dst->hint_col[o] = static_cast<size_t>(col) < np ? perm[col] : col;
                    if (dst->hint_val) std::memcpy(&dst->hint_val[o], &ent[k].y, sizeof(float));
                }
            }
        } else if (dst->hint_row_ptr) {
            std::memset(dst->hint_row_ptr, 0, (N + 1) * sizeof(int32_t));
        }
        if (g->norm_version >= 0 && (dst->degree || dst->scale)) {
            // operator arrays live in execution order; return them in node order
            std::vector<double> d(N);
            std::vector<float> sc(N);
            const size_t np = static_cast<size_t>(g->first_mvirt);
            std::vector<int32_t> perm(np);
            AHR_HIP(hipMemcpyAsync(d.data(), g->deg.p, N * sizeof(double), hipMemcpyDeviceToHost, s));
            AHR_HIP(hipMemcpyAsync(sc.data(), g->scale.p, N * sizeof(float), hipMemcpyDeviceToHost, s));
            AHR_HIP(hipMemcpyAsync(perm.data(), g->perm.p, np * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            AHR_HIP(hipStreamSynchronize(s));
            for (size_t r = 0; r < N; ++r) {
                size_t c = r < np ? static_cast<size_t>(perm[r]) : r;
                if (dst->degree) dst->degree[c] = d[r];
                if (dst->scale) dst->scale[c] = sc[r];
            }
        }
        if (g->norm_version >= 0 && dst->lambda_up) {
            double l = 0;
            AHR_HIP(hipMemcpyAsync(&l, g->lam.p, sizeof l, hipMemcpyDeviceToHost, s));
            AHR_HIP(hipStreamSynchronize(s));
            *dst->lambda_up = static_cast<float>(l);
        }
        AHR_HIP(hipStreamSynchronize(s));
        return AHR_OK;
    });
}

void ahr_graph_destroy(ahr_graph* h) {
    if (!h) return;
    try {
        delete reinterpret_cast<ahr::Graph*>(h);
    } catch (...) {
    }
    ahr::flush_frees();
}

ahr_status ahr_filter(ahr_graph* h, const ahr_filter_spec* spec, const float* in, float* out, int32_t ncols,
                      void* stream) {
    if (!h) return fail(AHR_EINVAL, "graph is NULL");
    ahr_status st;
    if ((st = check_spec(spec)) != AHR_OK) return st;
    if (!in || !out) return fail(AHR_EINVAL, "in/out is NULL");
    if (!ncols_ok(ncols)) return fail(AHR_EINVAL, "ncols must be 1, 2, 4 or 8");
    auto* gr = reinterpret_cast<ahr::Graph*>(h);
    if (!gr->has_hints) return fail(AHR_EINVAL, "graph has no hints yet: build with a placement or update_hints");
    size_t bytes = static_cast<size_t>(gr->n_inst) * ncols * sizeof(float);
    if (overlap(in, bytes, out, bytes)) return fail(AHR_EINVAL, "in and out overlap");
    return guarded([&]() -> ahr_status {
        ahr::ArenaScope arena_scope(gr->arena);
        gr->use_stream(as_stream(stream));
        ahr::run_filter(*gr, *spec, in, out, ncols, as_stream(stream));
        return AHR_OK;
    });
}

ahr_status ahr_gift(ahr_graph* h, const ahr_gift_spec* spec, const float* in, float* out, int32_t ncols,
                    void* stream) {
    if (!h) return fail(AHR_EINVAL, "graph is NULL");
    if (!spec) return fail(AHR_EINVAL, "GiFt spec is NULL");
    if (spec->nbands < 1 || spec->nbands > AHR_MAX_BANDS) return fail(AHR_EINVAL, "nbands in [1, 4]");
    for (int b = 0; b < spec->nbands; ++b) {
        if (spec->k[b] < 0 || spec->k[b] > 64) return fail(AHR_EINVAL, "k in [0, 64]");
        if (!std::isfinite(spec->alpha[b])) return fail(AHR_EINVAL, "alpha must be finite");
        if (!(spec->sigma[b] >= 0.f) || !std::isfinite(spec->sigma[b])) return fail(AHR_EINVAL, "sigma must be >= 0");
    }
    if (!in || !out) return fail(AHR_EINVAL, "in/out is NULL");
    if (!ncols_ok(ncols)) return fail(AHR_EINVAL, "ncols must be 1, 2, 4 or 8");
    auto* gr = reinterpret_cast<ahr::Graph*>(h);
    if (gr->hp.flags & (AHR_MACRO_HINTS | AHR_BIN_HINTS))
        return fail(AHR_EINVAL, "GiFt filters the netlist graph: build it with AHR_MACRO_HINTS and AHR_BIN_HINTS off");
    if (!gr->has_hints) return fail(AHR_EINVAL, "graph has no execution order yet: build it with a placement");
    size_t bytes = static_cast<size_t>(gr->n_inst) * ncols * sizeof(float);
    if (overlap(in, bytes, out, bytes)) return fail(AHR_EINVAL, "in and out overlap");
    return guarded([&]() -> ahr_status {
        ahr::ArenaScope arena_scope(gr->arena);
        gr->use_stream(as_stream(stream));
        ahr::run_gift(*gr, *spec, in, out, ncols, as_stream(stream));
        return AHR_OK;
    });
}

ahr_status ahr_graph_refine(ahr_graph* h, const ahr_filter_spec* spec, const float* g0, int32_t ncols, int32_t T_hint,
                      float gamma, float* out, void* stream) {
    if (!h) return fail(AHR_EINVAL, "graph is NULL");
    ahr_status st;
    if ((st = check_spec(spec)) != AHR_OK) return st;
    if (!g0 || !out) return fail(AHR_EINVAL, "g0/out is NULL");
    if (!ncols_ok(ncols) || ncols < 2) return fail(AHR_EINVAL, "ncols must be 2, 4 or 8");
    if (T_hint < 0) return fail(AHR_EINVAL, "T_hint must be >= 0");
    if (!(gamma >= 0.f && gamma <= 1.f)) return fail(AHR_EINVAL, "gamma in [0, 1]");
    auto* gr = reinterpret_cast<ahr::Graph*>(h);
    size_t bytes = static_cast<size_t>(gr->n_inst) * ncols * sizeof(float);
    if (g0 != out && overlap(g0, bytes, out, bytes)) return fail(AHR_EINVAL, "g0 and out partially overlap");
    return guarded([&]() -> ahr_status {
        ahr::ArenaScope arena_scope(gr->arena);
        hipStream_t s = as_stream(stream);
        gr->use_stream(s);
        size_t n = static_cast<size_t>(gr->n_inst) * ncols;
        if (T_hint == 0) {
            if (g0 != out) AHR_HIP(hipMemcpyAsync(out, g0, bytes, hipMemcpyDeviceToDevice, s));
            return AHR_OK;
        }
        gr->ga.ensure(n, s);
        gr->gb.ensure(n, s);
        gr->gt.ensure(n, s);
        const float* cur = g0;
        for (int r = 0; r < T_hint; ++r) {
            float* next = (r == T_hint - 1) ? out : ((r & 1) ? gr->gb.p : gr->ga.p);
            ahr::build_hints(*gr, cur, ncols, s, r > 0);     // later rounds: fixed macros stay put
            ahr::run_filter(*gr, *spec, cur, gr->gt.p, ncols, s);
            ahr::relax(*gr, cur, gr->gt.p, next, ncols, gamma, s);
            cur = next;
        }
        return AHR_OK;
    });
}

ahr_status ahr_refine(const ahr_netlist* nl, const ahr_hint_params* hp, const ahr_filter_spec* spec, const float* g0,
                      int32_t ncols, int32_t T_hint, float gamma, float* out, void* ws, size_t ws_bytes, void* stream) {
    ahr_status st;
    if ((st = check_netlist(nl)) != AHR_OK) return st;
    if ((st = check_hints(hp)) != AHR_OK) return st;
    if ((st = check_spec(spec)) != AHR_OK) return st;
    if (!g0 || !out) return fail(AHR_EINVAL, "g0/out is NULL");
    if (!ncols_ok(ncols) || ncols < 2) return fail(AHR_EINVAL, "ncols must be 2, 4 or 8");
    if (T_hint < 0) return fail(AHR_EINVAL, "T_hint must be >= 0");
    if (!(gamma >= 0.f && gamma <= 1.f)) return fail(AHR_EINVAL, "gamma in [0, 1]");
    size_t bytes = static_cast<size_t>(nl->n_inst) * ncols * sizeof(float);
    if (g0 != out && overlap(g0, bytes, out, bytes)) return fail(AHR_EINVAL, "g0 and out partially overlap");
    if (ws && ws_bytes < ahr::graph_workspace_floor(*nl, ncols))
        return fail(AHR_ENOMEM, "workspace too small for the netlist's sizes (ask ahr_graph_workspace_size)");
    return guarded([&]() -> ahr_status {
        hipStream_t s = as_stream(stream);
        ahr::Graph* gr = new_graph(nl, hp, nullptr, 0, ncols, ws, ws_bytes, s);
        struct Drop {
            ahr::Graph* g;
            ~Drop() { delete g; }
        } drop{gr};
        ahr::ArenaScope scope(gr->arena);
        if (T_hint == 0) {
            if (g0 != out) AHR_HIP(hipMemcpyAsync(out, g0, bytes, hipMemcpyDeviceToDevice, s));
            return AHR_OK;
        }
        const size_t n = static_cast<size_t>(gr->n_inst) * ncols;
        gr->ga.ensure(n, s);
        gr->gb.ensure(n, s);
        gr->gt.ensure(n, s);
        const float* cur = g0;
        for (int r = 0; r < T_hint; ++r) {
            float* next = (r == T_hint - 1) ? out : ((r & 1) ? gr->gb.p : gr->ga.p);
            ahr::build_hints(*gr, cur, ncols, s, r > 0);     // later rounds: fixed macros stay put
            ahr::run_filter(*gr, *spec, cur, gr->gt.p, ncols, s);
            ahr::relax(*gr, cur, gr->gt.p, next, ncols, gamma, s);
            cur = next;
        }
        return AHR_OK;
    });
}

ahr_status ahr_refine_learned(ahr_graph* h, const ahr_filter_spec* spec, const ahr_mlp* model, const float* g0,
                              int32_t ncols, int32_t T_hint, float gamma, float* out, int32_t* used_fallback,
                              void* stream) {
    if (!h) return fail(AHR_EINVAL, "graph is NULL");
    ahr_status st;
    if ((st = check_spec(spec)) != AHR_OK) return st;
    if (!model || !model->params) return fail(AHR_EINVAL, "model is NULL");
    if (!g0 || !out) return fail(AHR_EINVAL, "g0/out is NULL");
    if (!ncols_ok(ncols) || ncols < 2) return fail(AHR_EINVAL, "ncols must be 2, 4 or 8");
    if (T_hint < 0) return fail(AHR_EINVAL, "T_hint must be >= 0");
    if (!(gamma >= 0.f && gamma <= 1.f)) return fail(AHR_EINVAL, "gamma in [0, 1]");
    auto* gr = reinterpret_cast<ahr::Graph*>(h);
    size_t bytes = static_cast<size_t>(gr->n_inst) * ncols * sizeof(float);
    if (g0 != out && overlap(g0, bytes, out, bytes)) return fail(AHR_EINVAL, "g0 and out partially overlap");
    return guarded([&]() -> ahr_status {
        ahr::ArenaScope arena_scope(gr->arena);
        hipStream_t s = as_stream(stream);
        gr->use_stream(s);
        size_t n = static_cast<size_t>(gr->n_inst) * ncols;
        if (used_fallback) *used_fallback = model->validated ? 0 : 1;
        if (T_hint == 0) {
            if (g0 != out) AHR_HIP(hipMemcpyAsync(out, g0, bytes, hipMemcpyDeviceToDevice, s));
            return AHR_OK;
        }
        gr->ga.ensure(n, s);
        gr->gb.ensure(n, s);
        gr->gt.ensure(n, s);
        const float* cur = g0;
        for (int r = 0; r < T_hint; ++r) {
            float* next = (r == T_hint - 1) ? out : ((r & 1) ? gr->gb.p : gr->ga.p);
            ahr::build_hints(*gr, cur, ncols, s, r > 0);     // later rounds: fixed macros stay put
            if (model->validated)
                ahr::run_learned(*gr, *spec, model->params, model->beta, cur, gr->gt.p, ncols, nullptr, nullptr,
                                 nullptr, s);
            else
                ahr::run_filter(*gr, *spec, cur, gr->gt.p, ncols, s);
            ahr::relax(*gr, cur, gr->gt.p, next, ncols, gamma, s);
            cur = next;
        }
        return AHR_OK;
    });
}

ahr_status ahr_filter_learned(ahr_graph* h, const ahr_filter_spec* spec, const ahr_mlp* model, const float* in,
                              float* out, int32_t ncols, int32_t* used_fallback, void* stream) {
    if (!h) return fail(AHR_EINVAL, "graph is NULL");
    ahr_status st;
    if ((st = check_spec(spec)) != AHR_OK) return st;
    if (!model || !model->params) return fail(AHR_EINVAL, "model is NULL");
    if (!in || !out) return fail(AHR_EINVAL, "in/out is NULL");
    if (!ncols_ok(ncols)) return fail(AHR_EINVAL, "ncols must be 1, 2, 4 or 8");
    auto* gr = reinterpret_cast<ahr::Graph*>(h);
    if (!gr->has_hints) return fail(AHR_EINVAL, "graph has no hints yet: build with a placement or update_hints");
    size_t bytes = static_cast<size_t>(gr->n_inst) * ncols * sizeof(float);
    if (overlap(in, bytes, out, bytes)) return fail(AHR_EINVAL, "in and out overlap");
    return guarded([&]() -> ahr_status {
        ahr::ArenaScope arena_scope(gr->arena);
        hipStream_t s = as_stream(stream);
        gr->use_stream(s);
        if (!model->validated) {
            ahr::run_filter(*gr, *spec, in, out, ncols, s);
            if (used_fallback) *used_fallback = 1;
            return AHR_OK;
        }
        ahr::run_learned(*gr, *spec, model->params, model->beta, in, out, ncols, nullptr, nullptr, nullptr, s);
        if (used_fallback) *used_fallback = 0;
        return AHR_OK;
    });
}

ahr_status ahr_filter_features(ahr_graph* h, const ahr_filter_spec* spec, const float* in, int32_t ncols,
                               float* feats, float* hops, float* stats, void* stream) {
    if (!h) return fail(AHR_EINVAL, "graph is NULL");
    ahr_status st;
    if ((st = check_spec(spec)) != AHR_OK) return st;
    if (!in) return fail(AHR_EINVAL, "in is NULL");
    if (!ncols_ok(ncols)) return fail(AHR_EINVAL, "ncols must be 1, 2, 4 or 8");
    auto* gr = reinterpret_cast<ahr::Graph*>(h);
    if (!gr->has_hints) return fail(AHR_EINVAL, "graph has no hints yet: build with a placement or update_hints");
    return guarded([&]() -> ahr_status {
        ahr::ArenaScope arena_scope(gr->arena);
        static const float zero_beta[4] = {0.f, 0.f, 0.f, 0.f};
        ahr::DevBuf<float> p;
        hipStream_t s = as_stream(stream);
        gr->use_stream(s);
        p.ensure(AHR_MLP_NPARAM, s);
        AHR_HIP(hipMemsetAsync(p.p, 0, AHR_MLP_NPARAM * sizeof(float), s));
        ahr::run_learned(*gr, *spec, p.p, zero_beta, in, nullptr, ncols, feats, hops, stats, s);
        p.release(s);
        return AHR_OK;
    });
}

ahr_status ahr_mlp_forward(const float* params, const float* feats, int64_t n, float* o, void* stream) {
    if (!params || !o || (n > 0 && !feats)) return fail(AHR_EINVAL, "NULL argument");
    if (n < 0) return fail(AHR_EINVAL, "n must be >= 0");
    return guarded([&]() -> ahr_status {
        ahr::mlp_forward(params, feats, n, o, as_stream(stream));
        return AHR_OK;
    });
}

ahr_status ahr_mlp_loss_grad(const float* params, const float* feats, const float* target, int64_t n, float* grad,
                             double* loss, int32_t rounding, void* stream) {
    if (!params || !grad || (n > 0 && (!feats || !target))) return fail(AHR_EINVAL, "NULL argument");
    if (n < 0) return fail(AHR_EINVAL, "n must be >= 0");
    if (rounding != 0 && rounding != 1) return fail(AHR_EINVAL, "rounding must be 0 or 1");
    return guarded([&]() -> ahr_status {
        ahr::mlp_loss_grad(params, feats, target, n, grad, loss, rounding != 0, as_stream(stream));
        return AHR_OK;
    });
}

ahr_status ahr_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step, float lr, float beta1,
                        float beta2, float eps, void* stream) {
    if (!params || !m || !v || !grad) return fail(AHR_EINVAL, "NULL argument");
    if (step < 1) return fail(AHR_EINVAL, "step must be >= 1");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(AHR_EINVAL, "bad Adam hyper-parameters");
    return guarded([&]() -> ahr_status {
        ahr::mlp_adam(params, m, v, grad, step, lr, beta1, beta2, eps, as_stream(stream));
        return AHR_OK;
    });
}

ahr_status ahr_filter_tune(int32_t lanes_per_row, int32_t nontemporal) {
    if (lanes_per_row != 0) {
        if (lanes_per_row != AHR_HOP_ROW_BLOCK && lanes_per_row != AHR_HOP_AUTO &&
            (lanes_per_row < 1 || lanes_per_row > 64 || (lanes_per_row & (lanes_per_row - 1))))
            return fail(AHR_EINVAL,
                        "lanes_per_row must be a power of two in [1, 64], AHR_HOP_ROW_BLOCK, AHR_HOP_AUTO, "
                        "or 0 to keep it");
        ahr::g_hop_lanes = lanes_per_row;
    }
    if (nontemporal >= 0) ahr::g_hop_nt = nontemporal ? 1 : 0;
    return AHR_OK;
}

ahr_status ahr_filter_get_tune(int32_t* lanes_per_row, int32_t* nontemporal) {
    if (!lanes_per_row || !nontemporal) return fail(AHR_EINVAL, "NULL argument");
    *lanes_per_row = ahr::g_hop_lanes;
    *nontemporal = ahr::g_hop_nt;
    return AHR_OK;
}

ahr_status check_charge(const ahr_charge_params* cp) {
    if (!cp) return fail(AHR_EINVAL, "charge params are NULL");
    if (cp->model < AHR_CHARGE_GAUSSIAN || cp->model > AHR_CHARGE_SIGMOID) return fail(AHR_EINVAL, "unknown model");
    if (cp->T < 1 || cp->t < 0 || cp->t > cp->T) return fail(AHR_EINVAL, "need 0 <= t <= T, T >= 1");
    if (cp->nbx < 1 || cp->nby < 1 || cp->nbx > 4096 || cp->nby > 4096) return fail(AHR_EINVAL, "nbx, nby in [1, 4096]");
    if (cp->model == AHR_CHARGE_EXP && !(cp->sigma_factor > 0.f && std::isfinite(cp->sigma_factor)))
        return fail(AHR_EINVAL, "sigma_factor must be positive");
    if ((cp->model == AHR_CHARGE_LINEAR || cp->model == AHR_CHARGE_SIGMOID) &&
        !(cp->k_factor > 0.f && std::isfinite(cp->k_factor)))
        return fail(AHR_EINVAL, "k_factor must be positive");
    if (cp->model == AHR_CHARGE_GAUSSIAN) {
        if (!(cp->r0 > 0.f && cp->r0 < 1.f) || !(cp->r1 > 0.f && cp->r1 < 1.f)) return fail(AHR_EINVAL, "r0, r1 in (0, 1)");
        if (!(cp->beta_min > 0.f) || !(cp->beta_max > 0.f) || !std::isfinite(cp->beta_min) ||
            !std::isfinite(cp->beta_max))
            return fail(AHR_EINVAL, "beta_min, beta_max must be positive");
        if (!(cp->alpha0 >= 0.f && cp->alpha0 < cp->alpha1 && cp->alpha1 <= 1.f))
            return fail(AHR_EINVAL, "need 0 <= alpha0 < alpha1 <= 1");
    }
    return AHR_OK;
}

ahr_status ahr_charge_schedule(const ahr_charge_params* cp, double* param) {
    ahr_status st;
    if ((st = check_charge(cp)) != AHR_OK) return st;
    if (!param) return fail(AHR_EINVAL, "param is NULL");
    *param = ahr::charge_schedule(*cp);
    return AHR_OK;
}

ahr_status ahr_macro_charge(const ahr_netlist* nl, const float* g, int32_t ncols, const ahr_charge_params* cp,
                            double* bin_mass, void* stream) {
    ahr_status st;
    if ((st = check_netlist(nl)) != AHR_OK) return st;
    if ((st = check_charge(cp)) != AHR_OK) return st;
    if (!g || !bin_mass) return fail(AHR_EINVAL, "g/bin_mass is NULL");
    if (!ncols_ok(ncols) || ncols < 2) return fail(AHR_EINVAL, "ncols must be 2, 4 or 8");
    return guarded([&]() -> ahr_status {
        ahr::run_macro_charge(*nl, g, ncols, *cp, bin_mass, as_stream(stream));
        return AHR_OK;
    });
}

ahr_status ahr_hpwl(const ahr_netlist* nl, const float* g, int32_t ncols, double* out, void* stream) {
    ahr_status st;
    if ((st = check_netlist(nl)) != AHR_OK) return st;
    if (!g || !out) return fail(AHR_EINVAL, "g/out is NULL");
    if (ncols != 2 && ncols != 4 && ncols != 8) return fail(AHR_EINVAL, "ncols must be 2, 4 or 8");
    return guarded([&]() -> ahr_status {
        ahr::run_hpwl(*nl, g, ncols, out, as_stream(stream));
        return AHR_OK;
    });
}

}  // extern "C"
