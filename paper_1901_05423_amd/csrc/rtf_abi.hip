// rtf_abi.hip -- the extern "C" entry points of include/rtforest.h: argument
// checks, workspace layout and kernel launches.  Host code only.
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "rtf_internal.h"

using namespace rtf;

namespace {

constexpr int64_t MAX_I32 = 2147483647;

// Workspace layout of a forest of D distributions, n_total leaves, m_total cells.
struct Layout {
    size_t status, nodes, cells, dists, eoff, coff, tsum, tpre, dloc, tdist, dcnt, ditems, runs,
        total;
    int64_t ntiles;
};

// Per-tile arrays are sized for the smaller tile (more tiles) and the
// deferral list for whichever tile shape needs more slots, so that one
// workspace size serves every tile shape.
int64_t ntiles_of(int64_t n, int tile) { return (n + tile - 1) / tile; }

Layout make_layout(int32_t D, int64_t n, int64_t m) {
    Layout L;
    L.ntiles = ntiles_of(n, Tile1024::TILE);
    const int64_t defer_slots = std::max(L.ntiles * Tile1024::DEFER_CAP,
                                         ntiles_of(n, Tile2048::TILE) * Tile2048::DEFER_CAP);
    size_t o = 0;
    L.status = o;
    o = align256(o + 256);
    L.nodes = o;
    o = align256(o + sizeof(Node) * (size_t)n);
    L.cells = o;
    o = align256(o + sizeof(Cell) * (size_t)m);
    L.dists = o;
    o = align256(o + sizeof(Dist) * (size_t)D);
    L.eoff = o;
    o = align256(o + sizeof(int64_t) * (size_t)(D + 1));
    L.coff = o;
    o = align256(o + sizeof(int64_t) * (size_t)(D + 1));
    L.tsum = o;
    o = align256(o + sizeof(uint64_t) * (size_t)L.ntiles);
    L.tpre = o;
    o = align256(o + sizeof(uint64_t) * (size_t)(L.ntiles + 1));  // + the grand total
    L.dloc = o;
    o = align256(o + sizeof(uint64_t) * (size_t)D);
    L.tdist = o;
    o = align256(o + sizeof(int32_t) * (size_t)(L.ntiles + 2));
    L.dcnt = o;
    o = align256(o + sizeof(int32_t) * (size_t)L.ntiles);
    L.ditems = o;
    o = align256(o + sizeof(int32_t) * (size_t)defer_slots);
    L.runs = o;
    o = align256(o + sizeof(Run) * (size_t)run_cap(m));
    L.total = o;
    return L;
}

bool sizes_ok(int32_t D, int64_t n, int64_t m) {
    return D >= 1 && n >= D && m >= D && n <= MAX_I32 && m <= MAX_I32;
}

template <typename T>
bool aligned(const T *p, size_t a) {
    return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0;
}

rtf_status from_hip(hipError_t e) { return e == hipSuccess ? RTF_OK : RTF_ERR_HIP; }

rtf_status build_common(const uint32_t *w, const int64_t *elem_off, const int64_t *cell_off,
                        int32_t D, int64_t n, int64_t m, int32_t tile, void *ws, size_t ws_bytes,
                        hipStream_t st, rtf_forest *out) {
    if (!w || !ws || !out || !aligned(w, 4) || !aligned(ws, 256)) return RTF_ERR_INVALID_ARG;
    if (tile == 0) tile = TILE_DEFAULT;
    if (tile != Tile1024::TILE && tile != Tile2048::TILE) return RTF_ERR_INVALID_ARG;
    if (D > 1 && (!elem_off || !cell_off || !aligned(elem_off, 8) || !aligned(cell_off, 8)))
        return RTF_ERR_INVALID_ARG;
    if (n < 1 || m < 1 || D < 1) return RTF_ERR_INVALID_ARG;
    if (!sizes_ok(D, n, m)) return RTF_ERR_SIZE;
    const Layout L = make_layout(D, n, m);
    if (ws_bytes < L.total) return RTF_ERR_WORKSPACE;
    char *b = static_cast<char *>(ws);
    rtf_forest f;
    memset(&f, 0, sizeof f);
    f.D = D;
    f.tile = tile;
    f.n_total = n;
    f.m_total = m;
    f.nodes = b + L.nodes;
    f.cells = b + L.cells;
    f.dists = b + L.dists;
    f.elem_off = reinterpret_cast<int64_t *>(b + L.eoff);
    f.cell_off = reinterpret_cast<int64_t *>(b + L.coff);
    f.status = reinterpret_cast<uint32_t *>(b + L.status);
    f.scratch = b + L.tsum;
    f.scratch_bytes = L.total - L.tsum;

    BuildArgs a;
    a.w = w;
    a.src_elem_off = D > 1 ? elem_off : nullptr;
    a.src_cell_off = D > 1 ? cell_off : nullptr;
    a.elem_off = f.elem_off;
    a.cell_off = f.cell_off;
    a.D = D;
    a.n_total = n;
    a.m_total = m;
    a.tile = tile;
    a.ntiles = ntiles_of(n, tile);
    a.nodes = static_cast<Node *>(f.nodes);
    a.cells = static_cast<Cell *>(f.cells);
    a.dists = static_cast<Dist *>(f.dists);
    a.status = f.status;
    a.tile_sum = reinterpret_cast<uint64_t *>(b + L.tsum);
    a.tile_prefix = reinterpret_cast<uint64_t *>(b + L.tpre);
    a.dist_local = reinterpret_cast<uint64_t *>(b + L.dloc);
    a.tile_dist = reinterpret_cast<int32_t *>(b + L.tdist);
    a.defer_count = reinterpret_cast<int32_t *>(b + L.dcnt);
    a.defer_items = reinterpret_cast<int32_t *>(b + L.ditems);
    a.run_count = reinterpret_cast<uint64_t *>(b + L.status + 64);  // in the status block
    a.item_count = reinterpret_cast<uint32_t *>(b + L.status + 72);
    a.runs = reinterpret_cast<Run *>(b + L.runs);
    if (launch_build(a, st) != hipSuccess) return RTF_ERR_HIP;
    *out = f;
    return RTF_OK;
}

bool forest_ok(const rtf_forest *f) {
    return f && f->nodes && f->cells && f->dists && f->status && f->D >= 1 &&
           sizes_ok(f->D, f->n_total, f->m_total);
}

bool sample_args_ok(const uint64_t *u, int64_t S, const int32_t *idx, const double *x) {
    if (S < 0) return false;
    if (S == 0) return true;
    return u && idx && aligned(u, 8) && aligned(idx, 4) && (!x || aligned(x, 8));
}


}  // namespace

// The checks and launches of a backward pass whose scratch is w (shared by
// rtf_backward and the static-scratch variant).
rtf_status rtf::backward_enqueue(const rtf_forest *f, const int64_t *sample_off, const uint64_t *u,
                                 const int32_t *idx, const double *grad_x, int64_t S,
                                 const double *scale, double *grad_w, const BackwardScratch &w,
                                 hipStream_t stream) {
    if (!forest_ok(f) || !scale || !grad_w || S < 0) return RTF_ERR_INVALID_ARG;
    if (S > 0 && (!u || !idx || !grad_x)) return RTF_ERR_INVALID_ARG;
    if (f->D > 1 && !sample_off) return RTF_ERR_INVALID_ARG;
    if (!aligned(grad_w, 8) || !aligned(scale, 8)) return RTF_ERR_INVALID_ARG;
    return from_hip(launch_backward(static_cast<const Node *>(f->nodes),
                                    static_cast<const Dist *>(f->dists), f->elem_off, f->D,
                                    f->n_total, f->D > 1 ? sample_off : nullptr, u, idx, grad_x,
                                    S, scale, grad_w, w, stream));
}

extern "C" {

size_t rtf_workspace_bytes(int64_t n, int64_t m) {
    if (n < 1 || m < 1 || !sizes_ok(1, n, m)) return 0;
    return make_layout(1, n, m).total;
}

size_t rtf_workspace_bytes_batched(int32_t D, int64_t n_total, int64_t m_total) {
    if (!sizes_ok(D, n_total, m_total)) return 0;
    return make_layout(D, n_total, m_total).total;
}

rtf_status rtf_build(const uint32_t *w, int64_t n, int64_t m, void *ws, size_t ws_bytes,
                     hipStream_t stream, rtf_forest *out) {
    return build_common(w, nullptr, nullptr, 1, n, m, 0, ws, ws_bytes, stream, out);
}

rtf_status rtf_build_tiled(const uint32_t *w, int64_t n, int64_t m, int32_t tile, void *ws,
                           size_t ws_bytes, hipStream_t stream, rtf_forest *out) {
    if (tile == 0) return RTF_ERR_INVALID_ARG;
    return build_common(w, nullptr, nullptr, 1, n, m, tile, ws, ws_bytes, stream, out);
}

rtf_status rtf_build_batched_tiled(const uint32_t *w, const int64_t *elem_off,
                                   const int64_t *cell_off, int32_t D, int64_t n_total,
                                   int64_t m_total, int32_t tile, void *ws, size_t ws_bytes,
                                   hipStream_t stream, rtf_forest *out) {
    if (D < 1 || !elem_off || !cell_off || tile == 0) return RTF_ERR_INVALID_ARG;
    if (D == 1) {
        // offsets still copied so that the descriptor is self-contained
        if (!aligned(elem_off, 8) || !aligned(cell_off, 8)) return RTF_ERR_INVALID_ARG;
    }
    return build_common(w, elem_off, cell_off, D, n_total, m_total, tile, ws, ws_bytes, stream,
                        out);
}

rtf_status rtf_build_batched(const uint32_t *w, const int64_t *elem_off, const int64_t *cell_off,
                             int32_t D, int64_t n_total, int64_t m_total, void *ws,
                             size_t ws_bytes, hipStream_t stream, rtf_forest *out) {
    return rtf_build_batched_tiled(w, elem_off, cell_off, D, n_total, m_total, TILE_DEFAULT, ws,
                                   ws_bytes, stream, out);
}

size_t rtf_wide_workspace_bytes(int64_t n_total) {
    if (n_total < 1 || n_total > MAX_I32) return 0;
    return align256(sizeof(Wide) * (size_t)n_total);
}

rtf_status rtf_forest_widen(rtf_forest *f, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!forest_ok(f) || !ws || !aligned(ws, 256)) return RTF_ERR_INVALID_ARG;
    if (ws_bytes < rtf_wide_workspace_bytes(f->n_total)) return RTF_ERR_WORKSPACE;
    Wide *w = static_cast<Wide *>(ws);
    const hipError_t e = launch_widen(static_cast<const Node *>(f->nodes),
                                      static_cast<const Cell *>(f->cells),
                                      static_cast<const Dist *>(f->dists), f->elem_off, f->D,
                                      f->n_total, w, stream);
    if (e != hipSuccess) return RTF_ERR_HIP;
    f->wide = ws;
    return RTF_OK;
}

size_t rtf_balance_workspace_bytes(int64_t m_total) {
    if (m_total < 1 || m_total > MAX_I32) return 0;
    return 2 * align256(sizeof(int32_t) * (size_t)m_total);
}

rtf_status rtf_forest_balance(rtf_forest *f, void *ws, size_t ws_bytes, int64_t *h_rebuilt,
                              hipStream_t stream) {
    if (!forest_ok(f) || !ws || !aligned(ws, 256)) return RTF_ERR_INVALID_ARG;
    if (ws_bytes < rtf_balance_workspace_bytes(f->m_total)) return RTF_ERR_WORKSPACE;
    int32_t *deep = static_cast<int32_t *>(ws);
    int32_t *last = reinterpret_cast<int32_t *>(static_cast<char *>(ws) +
                                                align256(sizeof(int32_t) * (size_t)f->m_total));
    uint32_t *count = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(f->status) +
                                                   STATUS_BALANCE_OFFSET);
    if (launch_balance(static_cast<Node *>(f->nodes), static_cast<Cell *>(f->cells),
                       static_cast<const Dist *>(f->dists), f->elem_off, f->D, f->n_total,
                       f->m_total, deep, last, count, stream) != hipSuccess)
        return RTF_ERR_HIP;
    f->wide = nullptr;  // collapsed records, if any, describe the old trees
    if (h_rebuilt) {
        if (hipStreamSynchronize(stream) != hipSuccess) return RTF_ERR_HIP;
        uint32_t v = 0;
        if (hipMemcpy(&v, count, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return RTF_ERR_HIP;
        *h_rebuilt = (int64_t)v;
    }
    return RTF_OK;
}

rtf_status rtf_forest_depth(const rtf_forest *f, int32_t *h_depth, hipStream_t stream) {
    if (!forest_ok(f) || !h_depth) return RTF_ERR_INVALID_ARG;
    uint32_t *word = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(f->status) +
                                                  STATUS_DEPTH_OFFSET);
    if (launch_depth(static_cast<const Node *>(f->nodes), static_cast<const Cell *>(f->cells),
                     static_cast<const Dist *>(f->dists), f->elem_off, f->D, f->n_total, word,
                     stream) != hipSuccess)
        return RTF_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return RTF_ERR_HIP;
    uint32_t v = 0;
    if (hipMemcpy(&v, word, sizeof v, hipMemcpyDeviceToHost) != hipSuccess) return RTF_ERR_HIP;
    *h_depth = (int32_t)v;
    return RTF_OK;
}

rtf_status rtf_sample(const rtf_forest *f, const uint64_t *u, int64_t S, int32_t *out_idx,
                      double *out_x, hipStream_t stream) {
    if (!forest_ok(f) || !sample_args_ok(u, S, out_idx, out_x)) return RTF_ERR_INVALID_ARG;
    if (S == 0) return RTF_OK;
    return from_hip(launch_sample(static_cast<const Node *>(f->nodes),
                                  static_cast<const Wide *>(f->wide),
                                  static_cast<const Cell *>(f->cells),
                                  static_cast<const Dist *>(f->dists), nullptr, 1, f->n_total, f->m_total, u, S,
                                  out_idx, out_x, stream));
}

rtf_status rtf_sample_batched(const rtf_forest *f, const int64_t *sample_off, const uint64_t *u,
                              int64_t S, int32_t *out_idx, double *out_x, hipStream_t stream) {
    if (!forest_ok(f) || !sample_args_ok(u, S, out_idx, out_x)) return RTF_ERR_INVALID_ARG;
    if (!sample_off || !aligned(sample_off, 8)) return RTF_ERR_INVALID_ARG;
    if (S == 0) return RTF_OK;
    return from_hip(launch_sample(static_cast<const Node *>(f->nodes),
                                  static_cast<const Wide *>(f->wide),
                                  static_cast<const Cell *>(f->cells),
                                  static_cast<const Dist *>(f->dists), sample_off, f->D, f->n_total,
                                  f->m_total, u, S, out_idx, out_x, stream));
}

rtf_status rtf_sample_2d(const rtf_forest *f, const uint64_t *u2, int64_t S, int32_t *out_rc,
                         double *out_xy, hipStream_t stream) {
    if (!forest_ok(f) || f->D < 2 || !sample_args_ok(u2, S, out_rc, out_xy))
        return RTF_ERR_INVALID_ARG;
    // pairs are moved as 16-byte (u2, out_xy) and 8-byte (out_rc) vectors
    if (S > 0 && (!aligned(u2, 16) || !aligned(out_rc, 8) || (out_xy && !aligned(out_xy, 16))))
        return RTF_ERR_INVALID_ARG;
    if (S == 0) return RTF_OK;
    return from_hip(launch_sample_2d(static_cast<const Node *>(f->nodes),
                                     static_cast<const Wide *>(f->wide),
                                     static_cast<const Cell *>(f->cells),
                                     static_cast<const Dist *>(f->dists), f->D, f->n_total, u2, S,
                                     out_rc, out_xy, stream));
}

rtf_status rtf_sample_bsearch(const rtf_forest *f, const uint64_t *u, int64_t S,
                              int32_t *out_idx, double *out_x, hipStream_t stream) {
    if (!forest_ok(f) || !sample_args_ok(u, S, out_idx, out_x)) return RTF_ERR_INVALID_ARG;
    if (S == 0) return RTF_OK;
    return from_hip(launch_sample_bsearch(static_cast<const Node *>(f->nodes),
                                  static_cast<const Cell *>(f->cells),
                                          static_cast<const Dist *>(f->dists), false, u, S,
                                          out_idx, out_x, stream));
}

rtf_status rtf_sample_cutpoint_bsearch(const rtf_forest *f, const uint64_t *u, int64_t S,
                                       int32_t *out_idx, double *out_x, hipStream_t stream) {
    if (!forest_ok(f) || !sample_args_ok(u, S, out_idx, out_x)) return RTF_ERR_INVALID_ARG;
    if (S == 0) return RTF_OK;
    return from_hip(launch_sample_bsearch(static_cast<const Node *>(f->nodes),
                                  static_cast<const Cell *>(f->cells),
                                          static_cast<const Dist *>(f->dists), true, u, S,
                                          out_idx, out_x, stream));
}

rtf_status rtf_quantize_f32(const float *v, const int64_t *elem_off, int32_t D, int64_t n_total,
                            uint32_t *out, double *scale, uint32_t *status,
                            hipStream_t stream) {
    if (!v || !out || !scale || D < 1 || n_total < 1) return RTF_ERR_INVALID_ARG;
    if (!aligned(v, 4) || !aligned(out, 4) || !aligned(scale, 8) ||
        (status && !aligned(status, 4)))
        return RTF_ERR_INVALID_ARG;
    if (D > 1 && (!elem_off || !aligned(elem_off, 8))) return RTF_ERR_INVALID_ARG;
    if (n_total > MAX_I32 || n_total < D) return RTF_ERR_SIZE;
    return from_hip(
        launch_quantize(v, D > 1 ? elem_off : nullptr, D, n_total, out, scale, status, stream));
}

size_t rtf_backward_workspace_bytes(int32_t D, int64_t n_total) {
    if (D < 1 || n_total < D || n_total > MAX_I32) return 0;
    return backward_layout(D, n_total, nullptr, nullptr);
}

rtf_status rtf_backward(const rtf_forest *f, const int64_t *sample_off, const uint64_t *u,
                        const int32_t *idx, const double *grad_x, int64_t S, const double *scale,
                        double *grad_w, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (!forest_ok(f) || !ws || !aligned(ws, 256)) return RTF_ERR_INVALID_ARG;
    if (ws_bytes < rtf_backward_workspace_bytes(f->D, f->n_total)) return RTF_ERR_WORKSPACE;
    BackwardScratch w;
    backward_layout(f->D, f->n_total, static_cast<char *>(ws), &w);
    return backward_enqueue(f, sample_off, u, idx, grad_x, S, scale, grad_w, w, stream);
}

rtf_status rtf_check(const rtf_forest *f, hipStream_t stream) {
    if (!forest_ok(f)) return RTF_ERR_INVALID_ARG;
    if (hipStreamSynchronize(stream) != hipSuccess) return RTF_ERR_HIP;
    uint32_t s = 0;
    if (hipMemcpy(&s, f->status, sizeof s, hipMemcpyDeviceToHost) != hipSuccess)
        return RTF_ERR_HIP;
    for (int c = 1; c < 32; ++c)
        if (s & (1u << c)) return static_cast<rtf_status>(c);
    return RTF_OK;
}

rtf_status rtf_forest_export(const rtf_forest *f, void *h_nodes, void *h_cells, uint64_t *h_W,
                             hipStream_t stream) {
    if (!forest_ok(f)) return RTF_ERR_INVALID_ARG;
    if (hipStreamSynchronize(stream) != hipSuccess) return RTF_ERR_HIP;
    if (h_nodes && hipMemcpy(h_nodes, f->nodes, sizeof(Node) * (size_t)f->n_total,
                             hipMemcpyDeviceToHost) != hipSuccess)
        return RTF_ERR_HIP;
    if (h_cells && hipMemcpy(h_cells, f->cells, sizeof(Cell) * (size_t)f->m_total,
                             hipMemcpyDeviceToHost) != hipSuccess)
        return RTF_ERR_HIP;
    if (h_W) {
        Dist *tmp = static_cast<Dist *>(malloc(sizeof(Dist) * (size_t)f->D));
        if (!tmp) return RTF_ERR_INVALID_ARG;
        hipError_t e = hipMemcpy(tmp, f->dists, sizeof(Dist) * (size_t)f->D,
                                 hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            for (int32_t d = 0; d < f->D; ++d) h_W[d] = tmp[d].W;
        free(tmp);
        if (e != hipSuccess) return RTF_ERR_HIP;
    }
    return RTF_OK;
}

rtf_status rtf_forest_import(const void *h_nodes, const void *h_cells, const uint64_t *h_W,
                             const int64_t *h_elem_off, const int64_t *h_cell_off, int32_t D,
                             int64_t n_total, int64_t m_total, void *ws, size_t ws_bytes,
                             hipStream_t stream, rtf_forest *out) {
    if (!h_nodes || !h_cells || !h_W || !ws || !out || !aligned(ws, 256)) return RTF_ERR_INVALID_ARG;
    if (D > 1 && (!h_elem_off || !h_cell_off)) return RTF_ERR_INVALID_ARG;
    if (n_total < 1 || m_total < 1 || D < 1) return RTF_ERR_INVALID_ARG;
    if (!sizes_ok(D, n_total, m_total)) return RTF_ERR_SIZE;
    const Layout L = make_layout(D, n_total, m_total);
    if (ws_bytes < L.total) return RTF_ERR_WORKSPACE;
    // offsets and per-distribution parameters, as the build's scan kernel
    // derives them from the totals
    int64_t *eo = static_cast<int64_t *>(malloc(sizeof(int64_t) * (size_t)(D + 1)));
    int64_t *co = static_cast<int64_t *>(malloc(sizeof(int64_t) * (size_t)(D + 1)));
    Dist *dist = static_cast<Dist *>(malloc(sizeof(Dist) * (size_t)D));
    uint32_t *status = static_cast<uint32_t *>(calloc(64, sizeof(uint32_t)));  // the 256-byte status block
    rtf_status rc = RTF_OK;
    if (!eo || !co || !dist || !status) rc = RTF_ERR_INVALID_ARG;
    uint64_t G = 0;
    for (int32_t q = 0; rc == RTF_OK && q <= D; ++q) {
        eo[q] = D > 1 ? h_elem_off[q] : (q ? n_total : 0);
        co[q] = D > 1 ? h_cell_off[q] : (q ? m_total : 0);
        if (q > 0 && (eo[q] <= eo[q - 1] || co[q] <= co[q - 1])) rc = RTF_ERR_INVALID_ARG;
    }
    if (rc == RTF_OK && (eo[0] != 0 || co[0] != 0 || eo[D] != n_total || co[D] != m_total))
        rc = RTF_ERR_INVALID_ARG;
    for (int32_t d = 0; rc == RTF_OK && d < D; ++d) {
        Dist P;
        memset(&P, 0, sizeof P);
        P.W = h_W[d];
        P.G0 = G;
        G += P.W;
        P.eo = eo[d];
        P.n = eo[d + 1] - eo[d];
        P.co = co[d];
        P.m = co[d + 1] - co[d];
        if (P.W == 0) {
            P.flags = DIST_ZERO;
            status[0] |= status_bit(RTF_ERR_ZERO_TOTAL);
        } else {
            P.s = (uint32_t)clz64(P.W);
            P.v = reciprocal_2by1(P.W << P.s);
        }
        if (P.m > 1 && (P.m & (P.m - 1)) == 0)
            P.flags |= (uint32_t)(64 - __builtin_ctzll((uint64_t)P.m)) << DIST_SHIFT_BIT;
        dist[d] = P;
    }
    char *b = static_cast<char *>(ws);
    rtf_forest f;
    memset(&f, 0, sizeof f);
    f.D = D;
    f.tile = TILE_DEFAULT;
    f.n_total = n_total;
    f.m_total = m_total;
    f.nodes = b + L.nodes;
    f.cells = b + L.cells;
    f.dists = b + L.dists;
    f.elem_off = reinterpret_cast<int64_t *>(b + L.eoff);
    f.cell_off = reinterpret_cast<int64_t *>(b + L.coff);
    f.status = reinterpret_cast<uint32_t *>(b + L.status);
    f.scratch = b + L.tsum;
    f.scratch_bytes = L.total - L.tsum;
    if (rc == RTF_OK) {
        const struct {
            void *dst;
            const void *src;
            size_t bytes;
        } copies[] = {{f.nodes, h_nodes, sizeof(Node) * (size_t)n_total},
                      {f.cells, h_cells, sizeof(Cell) * (size_t)m_total},
                      {f.dists, dist, sizeof(Dist) * (size_t)D},
                      {f.elem_off, eo, sizeof(int64_t) * (size_t)(D + 1)},
                      {f.cell_off, co, sizeof(int64_t) * (size_t)(D + 1)},
                      {f.status, status, 256}};
        for (const auto &c : copies)
            if (rc == RTF_OK &&
                hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
                rc = RTF_ERR_HIP;
        // the host staging buffers must outlive the copies
        if (hipStreamSynchronize(stream) != hipSuccess && rc == RTF_OK) rc = RTF_ERR_HIP;
    }
    free(eo);
    free(co);
    free(dist);
    free(status);
    if (rc == RTF_OK) *out = f;
    return rc;
}

const char *rtf_status_string(rtf_status s) {
    switch (s) {
    case RTF_OK: return "RTF_OK";
    case RTF_ERR_INVALID_ARG: return "RTF_ERR_INVALID_ARG";
    case RTF_ERR_SIZE: return "RTF_ERR_SIZE";
    case RTF_ERR_WORKSPACE: return "RTF_ERR_WORKSPACE";
    case RTF_ERR_HIP: return "RTF_ERR_HIP";
    case RTF_ERR_ZERO_TOTAL: return "RTF_ERR_ZERO_TOTAL";
    case RTF_ERR_VALUE: return "RTF_ERR_VALUE";
    }
    return "RTF_ERR_UNKNOWN";
}

}  // extern "C"
