// md_api.hip -- host side of the C ABI declared in include/md.h.
//
// Owns the device buffers of a context (one box or an ensemble), validates
// arguments synchronously, enqueues the kernels of md_kernels.hip on the
// context stream, and turns device-side status words into md_status codes at
// the few synchronizing points (end of an md_step call, energies, diagnostics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "md.h"
#include "md_internal.h"

using namespace mdg;

namespace {

constexpr int kChunk = 200;      // steps enqueued between status checks
constexpr int64_t kTileMinN = 1 << 23;  // FP32-mixed boxes from this size take row tiles by default
constexpr int kGraphSteps = 8;   // continuing steps per captured graph

// Message of the last failed md_create / md_batch_create (no context exists then).
thread_local std::string g_create_err;

const char* kStatusStr[] = {"MD_OK", "MD_EINVAL", "MD_ENOMEM", "MD_EHIP", "MD_ENUMERIC", "MD_ESTATE", "MD_ELIST"};

}  // namespace

struct md_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int nbox = 0;
    md_params prm{};               // shared fields (box 0's record)
    std::vector<md_params> boxes;  // per box as given (box lengths change on rescale)
    std::vector<BoxGeom> geom;
    int64_t ntotal = 0;
    int32_t nslot = 0, nwave = 0, ntile = 0, nrows = 0;
    bool tile_fallback = false;    // a row tile overflowed its staging capacity: gather format from then on
    bool prefer_gather = false;    // gather format over row tiles: by size at creation, or md_autotune's choice
    double cell_scale = 0.0;       // > 0: cell side bound chosen by md_autotune (else the boxes' own)
    Params P{};
    Dev D{};
    // device allocations not reachable through D
    double* bk_pos = nullptr;    // caller-order copy of the state while md_autotune re-lays
    double* bk_vel = nullptr;    // the grid (allocated on its first call)
    double* dscratch = nullptr;  // nbox doubles (scale factors)
    BoxState* st_h = nullptr;    // pinned mirror of the box states
    int64_t list_alloc = 0;      // entries allocated in D.list
    bool have_state = false, have_cells = false, have_list = false, have_F = false;
    md_status sticky = MD_OK;
    std::string err;
    int64_t steps = 0, regrows = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev_force, ev_rebuild;  // start/stop pairs
    // captured step graphs (MD_F_GRAPH): kGraphSteps and 1 continuing steps
    hipGraphExec_t graph_many = nullptr, graph_one = nullptr;
    double force_ms = 0.0, rebuild_ms = 0.0;
    int64_t force_n = 0, rebuild_n = 0;
    // bubble analysis work buffers (md_bubbles), bw_alloc subcells each
    BubbleWork bw{};
    int64_t bw_alloc = 0;
};

namespace {

md_status fail(md_ctx* c, md_status s, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
        if (s == MD_EHIP) c->sticky = MD_EHIP;
    }
    return s;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((ctx), e_ == hipErrorOutOfMemory ? MD_ENOMEM : MD_EHIP, "%s: %s (%s:%d)", \
                        #call, hipGetErrorString(e_), __FILE__, __LINE__);                       \
    } while (0)

#define LAUNCHCHK(ctx)                                                                     \
    do {                                                                                   \
        hipError_t e_ = hipGetLastError();                                                 \
        if (e_ != hipSuccess)                                                              \
            return fail((ctx), MD_EHIP, "kernel launch: %s (%s:%d)", hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                               \
    } while (0)

template <typename T>
md_status dalloc(md_ctx* c, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, MD_ENOMEM, "hipMalloc of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(e));
    }
    return MD_OK;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

void drop_graphs(md_ctx* c);

// Argument checks of md_create / md_batch_create (no device work).
md_status validate(const md_params* b, int32_t nbox, std::string& why) {
    char buf[256];
    if (!b || nbox < 1) {
        why = "null params or nbox < 1";
        return MD_EINVAL;
    }
    int64_t slots = 0;
    for (int32_t i = 0; i < nbox; ++i) {
        const md_params& p = b[i];
        auto bad = [&](const char* what) {
            snprintf(buf, sizeof buf, "box %d: %s", i, what);
            why = buf;
            return MD_EINVAL;
        };
        if (p.n < 2) return bad("n < 2");
        if (!finite_pos(p.rc)) return bad("rc must be finite and > 0");
        if (!(std::isfinite(p.skin) && p.skin >= 0.0)) return bad("skin must be finite and >= 0");
        if (!finite_pos(p.dt)) return bad("dt must be finite and > 0");
        if (!finite_pos(p.mass)) return bad("mass must be finite and > 0");
        if (p.precision != MD_PREC_FP64 && p.precision != MD_PREC_FP32_MIXED) return bad("unknown precision");
        if (p.cutoff < MD_CUT_EQ1 || p.cutoff > MD_CUT_RAW) return bad("unknown cutoff scheme");
        if (p.rebuild < MD_REBUILD_DUTC || p.rebuild > MD_REBUILD_NEVER) return bad("unknown rebuild policy");
        if (p.flags &
            ~(uint32_t)(MD_F_VERIFY_LIST | MD_F_GRAPH | MD_F_TILE_ON | MD_F_TILE_OFF | MD_F_FAST_RCP | MD_F_HALF_LIST))
            return bad("unknown flag bits");
        if ((p.flags & MD_F_HALF_LIST) && (p.flags & (MD_F_VERIFY_LIST | MD_F_TILE_ON)))
            return bad("MD_F_HALF_LIST does not combine with MD_F_VERIFY_LIST or MD_F_TILE_ON");
        if ((p.flags & MD_F_HALF_LIST) && p.threads_per_key > 1)
            return bad("MD_F_HALF_LIST takes one lane per key (threads_per_key 0 or 1)");
        if ((p.flags & MD_F_FAST_RCP) && p.precision != MD_PREC_FP64)
            return bad("MD_F_FAST_RCP applies to the FP64 path only");
        if ((p.flags & MD_F_TILE_ON) && (p.flags & MD_F_TILE_OFF)) return bad("MD_F_TILE_ON with MD_F_TILE_OFF");
        if ((p.flags & MD_F_TILE_ON) && p.threads_per_key > 1)
            return bad("MD_F_TILE_ON takes one lane per key (threads_per_key 0 or 1)");
        if (!(p.threads_per_key == 0 || p.threads_per_key == 1 || p.threads_per_key == 2 ||
              p.threads_per_key == 4 || p.threads_per_key == 8))
            return bad("threads_per_key must be 0, 1, 2, 4 or 8");
        if (p.list_cap < 0 || p.list_cap > 4096) return bad("list_cap must be in [0, 4096]");
        for (int k = 0; k < 5; ++k)
            if (p.reserved[k]) return bad("reserved fields must be zero");
        if (!(p.cell_scale == 0.0 || (p.cell_scale >= 1.0 && p.cell_scale <= 2.0)))
            return bad("cell_scale must be 0 or in [1, 2]");
        const double rl = p.rc + p.skin;
        for (int a = 0; a < 3; ++a) {
            if (!finite_pos(p.box[a])) return bad("box lengths must be finite and > 0");
            if (p.box[a] < 3.0 * rl) return bad("box side below 3 * (rc + skin)");
            if (std::floor(p.box[a] / rl) > kMaxCellsPerAxis) return bad("more than 1023 cells per axis");
        }
        if (i > 0) {
            const md_params& q = b[0];
            if (p.rc != q.rc || p.skin != q.skin || p.dt != q.dt || p.mass != q.mass ||
                p.precision != q.precision || p.cutoff != q.cutoff || p.rebuild != q.rebuild ||
                p.flags != q.flags || p.threads_per_key != q.threads_per_key || p.list_cap != q.list_cap ||
                p.cell_scale != q.cell_scale)
                return bad("rc, skin, dt, mass, precision, cutoff, rebuild, flags, threads_per_key, "
                           "list_cap and cell_scale must agree across boxes");
        }
        slots += (p.n + kWave - 1) / kWave * kWave;
        if (slots > (int64_t)kIdxMask + 1) return bad("more than 2^27 particle slots in total");
    }
    return MD_OK;
}

void lj_coeffs(double rc, int mode, double* c2, double* c0) {
    // Eq. (1): V/4 = r^-12 - r^-6 + c2 r^2 + c0 with V(rc) = V'(rc) = 0.
    const double s = 1.0 / (rc * rc), s3 = s * s * s;
    if (mode == MD_CUT_EQ1) {
        *c2 = 6.0 * s3 * s3 * s - 3.0 * s3 * s;
        *c0 = -7.0 * s3 * s3 + 4.0 * s3;
    } else if (mode == MD_CUT_SHIFT) {
        *c2 = 0.0;
        *c0 = s3 - s3 * s3;
    } else {
        *c2 = 0.0;
        *c0 = 0.0;
    }
}

// Box geometry: cell grid n = floor(L / r_list) per axis, inv = n / L, cs = L / n,
// and the placement of each box's cells and slots in the shared arrays.
// Cell side lower bound as a multiple of r_list: md_autotune's choice, else the
// parameters' own (0 = 1).
double cell_scale_of(const md_ctx* c) {
    if (c->cell_scale > 0.0) return c->cell_scale;
    return c->prm.cell_scale > 0.0 ? c->prm.cell_scale : 1.0;
}

void layout(md_ctx* c) {
    const double rl = c->prm.rc + c->prm.skin, side = rl * cell_scale_of(c);
    c->geom.assign(c->nbox, BoxGeom{});
    int32_t slot = 0, tile = 0, rows = 0;
    int64_t id = 0;
    for (int b = 0; b < c->nbox; ++b) {
        BoxGeom& g = c->geom[b];
        const md_params& p = c->boxes[b];
        double csmax = 0.0;
        for (int a = 0; a < 3; ++a) {
            g.L[a] = p.box[a];
            // cells of side >= side (>= r_list): at least 3 per axis, which the box
            // size bound L >= 3 r_list always allows
            g.n[a] = std::max(3, (int32_t)std::floor(p.box[a] / side));
            g.inv[a] = (double)g.n[a] / p.box[a];
            g.cs[a] = p.box[a] / (double)g.n[a];
            csmax = std::max(csmax, g.cs[a]);
        }
        // fixed-point unit: a power of two, one cell side = 2^27 .. 2^28 units
        int e;
        (void)std::frexp(csmax, &e);  // csmax in [2^(e-1), 2^e)
        g.ucs = std::ldexp(1.0, kUnitBits - e);
        for (int a = 0; a < 3; ++a) {
            g.uoff[a] = (int32_t)std::lrint(g.cs[a] * g.ucs);
            g.nuoff[a] = (int32_t)(uint32_t)((uint64_t)g.n[a] * (uint64_t)(uint32_t)g.uoff[a]);
        }
        g.lam = (float)std::ldexp(1.0, e - kUnitBits);
        g.lam2inv = (float)(g.ucs * g.ucs);
        g.rc2u = (float)(p.rc * p.rc * g.ucs * g.ucs);
        g.ncell = g.n[0] * g.n[1] * g.n[2];
        const int64_t divs[3] = {g.n[0], g.n[1], (int64_t)g.n[0] * g.n[1]};
        for (int k = 0; k < 3; ++k) {
            int l = 0;
            while (((int64_t)1 << l) < divs[k]) ++l;  // n >= 3: l >= 2
            g.dmul[k] = (uint32_t)((((uint64_t)1) << (30 + l)) / (uint64_t)divs[k] + 1);
            g.dshr[k] = l - 2;
        }
        g.ntile = (g.ncell + kTile - 1) / kTile;
        g.tile_off = tile;
        g.cell_off = tile * kTile;
        tile += g.ntile;
        g.npart = (int32_t)p.n;
        g.nslot = (int32_t)((p.n + kWave - 1) / kWave * kWave);
        g.slot_off = slot;
        slot += g.nslot;
        g.id_off = (int32_t)id;
        id += p.n;
        g.row_off = rows;
        rows += g.n[1] * g.n[2];
    }
    c->nrows = rows;
    c->nslot = slot;
    c->nwave = slot / kWave;
    c->ntile = tile;
    c->ntotal = id;
}

// Estimated longest full list: 1.5x the mean at the densest box, plus margin.
int32_t estimate_cap(const md_ctx* c) {
    const double rl = c->prm.rc + c->prm.skin;
    double mean = 0.0;
    for (int b = 0; b < c->nbox; ++b) {
        const md_params& p = c->boxes[b];
        const double rho = (double)p.n / (p.box[0] * p.box[1] * p.box[2]);
        mean = std::max(mean, rho * 4.0 / 3.0 * M_PI * rl * rl * rl);
    }
    // a half list holds half the partners on average, but its lengths spread more
    // (a cell's first particle lists its whole cell, the last none of it)
    if (c->prm.flags & MD_F_HALF_LIST) return (int32_t)std::ceil(0.75 * mean) + 24;
    return (int32_t)std::ceil(1.5 * mean) + 16;
}

md_status upload_geometry(md_ctx* c) {
    HIPCHK(c, hipMemcpyAsync(c->D.geom, c->geom.data(), sizeof(BoxGeom) * c->nbox, hipMemcpyHostToDevice,
                             c->stream));
    std::vector<int32_t> wb(c->nwave), tb(c->ntile), rb(c->nrows);
    for (int b = 0; b < c->nbox; ++b) {
        const BoxGeom& g = c->geom[b];
        for (int w = 0; w < g.nslot / kWave; ++w) wb[g.slot_off / kWave + w] = b;
        for (int t = 0; t < g.ntile; ++t) tb[g.tile_off + t] = b;
        for (int r = 0; r < g.n[1] * g.n[2]; ++r) rb[g.row_off + r] = b;
    }
    std::vector<double4> dsh(27 * c->nbox);
    for (int b = 0; b < c->nbox; ++b) {
        const BoxGeom& g = c->geom[b];
        for (int z = -1; z <= 1; ++z)
            for (int y = -1; y <= 1; ++y)
                for (int x = -1; x <= 1; ++x) {
                    const int code = (z + 1) * 9 + (y + 1) * 3 + (x + 1);
                    // code = periodic image r; the FP64 force subtracts r * L.
                    dsh[b * 27 + code] = make_double4(x * g.L[0], y * g.L[1], z * g.L[2], 0.0);
                }
    }
    HIPCHK(c, hipMemcpyAsync(c->D.wave_box, wb.data(), sizeof(int32_t) * wb.size(), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->D.tile_box, tb.data(), sizeof(int32_t) * tb.size(), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->D.row_box, rb.data(), sizeof(int32_t) * rb.size(), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->D.dshift, dsh.data(), sizeof(double4) * dsh.size(), hipMemcpyHostToDevice,
                             c->stream));
    // the vectors above are pageable: finish the copies before they go away
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MD_OK;
}

md_status alloc_cells(md_ctx* c) {
    drop_graphs(c);
    dfree(c->D.tile_box);
    dfree(c->D.cell_cnt);
    dfree(c->D.cell_start);
    dfree(c->D.tile_sum);
    dfree(c->D.tile_pref);
    dfree(c->D.tile_need);
    dfree(c->D.rtile);
    dfree(c->D.row_box);
    dfree(c->D.row_nt);
    dfree(c->D.row_t0);
    dfree(c->D.cell_rt);
    dfree(c->D.rt_tmp);
    dfree(c->D.rt_delta);
    dfree(c->D.ke_part);
    dfree(c->D.pe_part);
    dfree(c->D.vir_part);
    dfree(c->D.red);
    md_status s;
    const size_t ncellpad = (size_t)c->ntile * kTile;
    // energy partials: per list wavefront, or per row tile (at most one per cell)
    const size_t nparts = std::max((size_t)c->nwave * 8, ncellpad);
    if ((s = dalloc(c, &c->D.rtile, ncellpad)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.row_box, c->nrows)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.row_nt, c->nrows)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.row_t0, c->nrows)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.cell_rt, ncellpad)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.rt_tmp, ncellpad)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.rt_delta, ncellpad * 27)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.ke_part, nparts)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.pe_part, nparts)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.vir_part, nparts)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.red, (size_t)c->nbox * c->P.redcap * 3)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.tile_box, c->ntile)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.cell_cnt, (size_t)c->ntile * kTile)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.cell_start, (size_t)c->ntile * kTile)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.tile_sum, c->ntile)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.tile_pref, c->ntile)) != MD_OK) return s;
    if ((s = dalloc(c, &c->D.tile_need, c->ntile)) != MD_OK) return s;
    return MD_OK;
}

// Captured graphs bake in kernel arguments (buffer pointers, sizes): drop them
// whenever those change.
void drop_graphs(md_ctx* c) {
    if (c->graph_many) (void)hipGraphExecDestroy(c->graph_many);
    if (c->graph_one) (void)hipGraphExecDestroy(c->graph_one);
    c->graph_many = c->graph_one = nullptr;
}

md_status alloc_list(md_ctx* c, int32_t cap) {
    drop_graphs(c);
    const int tpk = c->P.tpk;
    cap = (cap + 8 * tpk - 1) / (8 * tpk) * (8 * tpk);  // rows = cap / tpk is a multiple of 8
    dfree(c->D.list);
    const int64_t entries = (int64_t)c->nslot * cap;
    md_status s = dalloc(c, &c->D.list, (size_t)entries);
    if (s != MD_OK) return s;
    c->list_alloc = entries;
    c->P.cap = cap;
    c->P.rows = cap / tpk;
    return MD_OK;
}

// A larger list during stepping: the entries move to the new layout, so the boxes
// that do not rebuild at the step the overflow stopped keep their lists.
md_status grow_list_keeping(md_ctx* c, int32_t cap) {
    uint16_t* old = c->D.list;
    const int32_t old_rows = c->P.rows;
    c->D.list = nullptr;
    md_status s = alloc_list(c, cap);  // frees nothing now: the old buffer is held here
    if (s != MD_OK) {
        c->D.list = old;
        return s;
    }
    launch_list_relayout(c->D, c->P, old, old_rows, c->stream);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(old);
    return MD_OK;
}

void params_refresh(md_ctx* c) {
    Params& P = c->P;
    const md_params& p = c->prm;
    double c2, c0;
    lj_coeffs(p.rc, p.cutoff, &c2, &c0);
    const double rl = p.rc + p.skin;
    P.rc2 = p.rc * p.rc;
    P.rl2 = rl * rl;
    P.c2 = c2;
    P.c0 = c0;
    P.dt = p.dt;
    P.h = p.dt / (2.0 * p.mass);
    P.mass = p.mass;
    P.skin = p.skin;
    P.rc2f = (float)P.rc2;
    P.irc2f = (float)(1.0 / P.rc2);
    P.clamp = p.cutoff == MD_CUT_EQ1 ? 1 : 0;
    P.c2f = (float)c2;
    P.c0f = (float)c0;
    P.policy = p.rebuild;
    P.nbox = c->nbox;
    P.nwave = c->nwave;
    P.ntile = c->ntile;
    P.precision = p.precision;
    P.half = (p.flags & MD_F_HALF_LIST) ? 1 : 0;
    // Row tiles (full list, one lane per key): the force pass reads every partner from
    // LDS; the gather format serves the other layouts, the sizes where it is faster, and
    // boxes whose cells are too crowded for a tile's staging capacity.
    P.tile = !P.half && P.tpk == 1 && !(p.flags & MD_F_TILE_OFF) && !c->tile_fallback && !c->prefer_gather ? 1 : 0;
    P.recb = p.precision == MD_PREC_FP64 ? 24 : 12;  // FP64 x, y, z or three fixed-point ints
    P.kt = kRtBlock;
    P.scap = kStageCap;
    P.nrows = c->nrows;
    P.maxslot = 0;
    P.maxcell = 0;
    for (const BoxGeom& g : c->geom) {
        P.maxslot = std::max(P.maxslot, g.nslot);
        P.maxcell = std::max(P.maxcell, g.ncell);
    }
    P.redcap = (std::max(P.maxslot / kWave * 8, P.maxcell) + kRedSeg - 1) / kRedSeg;
    // Row-tile force kernel: one resident round of blocks, each looping over the tiles
    // (block k takes tiles k, k + grid, ...).  With the XCD-aware order each XCD then
    // sweeps the same band of rows plane after plane, so the rows it stages stay in its
    // L2; a grid of one block per tile measured 16% slower at 32M particles.
    if (P.tgrid <= 0) {
        hipDeviceProp_t prop;
        int cus = 256;
        if (hipGetDeviceProperties(&prop, c->device) == hipSuccess && prop.multiProcessorCount > 0)
            cus = prop.multiProcessorCount;
        P.tgrid = cus * rowtile_blocks_per_cu(P);
    }
    P.fastrcp = (p.flags & MD_F_FAST_RCP) ? 1 : 0;
}

void free_all(md_ctx* c) {
    drop_graphs(c);
    Dev& D = c->D;
    dfree(D.geom);
    dfree(D.st);
    dfree(D.any);
    dfree(D.halt);
    dfree(D.wave_box);
    dfree(D.tile_box);
    for (int k = 0; k < 2; ++k) {
        dfree(D.q[k]);
        dfree(D.u[k]);
        dfree(D.vx[k]);
        dfree(D.vy[k]);
        dfree(D.vz[k]);
        dfree(D.id[k]);
    }
    dfree(D.qb);
    dfree(D.fx);
    dfree(D.fy);
    dfree(D.fz);
    dfree(D.cnt);
    dfree(D.list);
    dfree(D.cell_tmp);
    dfree(D.ticket);
    dfree(D.perm);
    dfree(D.cell_cnt);
    dfree(D.cell_start);
    dfree(D.tile_sum);
    dfree(D.tile_pref);
    dfree(D.tile_need);
    dfree(D.rtile);
    dfree(D.row_box);
    dfree(D.row_nt);
    dfree(D.row_t0);
    dfree(D.ntiles);
    dfree(D.box_t0);
    dfree(D.cell_rt);
    dfree(D.rt_tmp);
    dfree(D.rt_delta);
    dfree(D.vmax_s);
    dfree(D.disp_s);
    dfree(D.ke_part);
    dfree(D.pe_part);
    dfree(D.vir_part);
    dfree(D.red);
    dfree(D.dshift);
    dfree(D.series_ke);
    dfree(D.series_pe);
    dfree(D.series_vir);
    dfree(D.series_th);
    dfree(c->bk_pos);
    dfree(c->bk_vel);
    dfree(c->dscratch);
    dfree(c->bw.cnt);
    dfree(c->bw.par);
    dfree(c->bw.lab);
    dfree(c->bw.size);
    dfree(c->bw.roots);
    dfree(c->bw.flag);
    c->bw_alloc = 0;
    if (c->st_h) (void)hipHostFree(c->st_h);
    c->st_h = nullptr;
    for (hipEvent_t e : c->ev_force) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_rebuild) (void)hipEventDestroy(e);
    c->ev_force.clear();
    c->ev_rebuild.clear();
}

md_status alloc_all(md_ctx* c) {
    Dev& D = c->D;
    const size_t ns = c->nslot;
    md_status s;
#define A(ptr, n)                                        \
    do {                                                 \
        if ((s = dalloc(c, &(ptr), (n))) != MD_OK) return s; \
    } while (0)
    A(D.geom, c->nbox);
    A(D.st, c->nbox);
    A(D.any, 1);
    A(D.halt, 1);
    A(D.wave_box, c->nwave);
    for (int k = 0; k < 2; ++k) {
        A(D.q[k], ns);
        if (c->prm.precision == MD_PREC_FP32_MIXED) A(D.u[k], 3 * ns);
        A(D.vx[k], ns);
        A(D.vy[k], ns);
        A(D.vz[k], ns);
        A(D.id[k], ns);
    }
    if (c->prm.rebuild == MD_REBUILD_DISPLACEMENT) A(D.qb, ns);
    A(D.fx, ns);
    A(D.fy, ns);
    A(D.fz, ns);
    A(D.cnt, ns);
    A(D.cell_tmp, ns);
    A(D.ticket, ns);
    A(D.perm, ns);
    A(D.vmax_s, (size_t)c->nbox * kStripes * kStripeStride);
    A(D.disp_s, (size_t)c->nbox * kStripes * kStripeStride);
    A(D.ntiles, 2);
    A(D.box_t0, (size_t)c->nbox + 1);
    A(D.dshift, (size_t)27 * c->nbox);
    A(D.series_ke, (size_t)kMaxSeries * c->nbox);
    A(D.series_pe, (size_t)kMaxSeries * c->nbox);
    A(D.series_vir, (size_t)kMaxSeries * c->nbox);
    A(D.series_th, (size_t)kMaxSeries * c->nbox);
    A(c->dscratch, (size_t)c->nbox);
#undef A
    if ((s = alloc_cells(c)) != MD_OK) return s;
    HIPCHK(c, hipMemsetAsync(D.any, 0, sizeof(int32_t), c->stream));
    HIPCHK(c, hipMemsetAsync(D.halt, 0, sizeof(int32_t), c->stream));
    HIPCHK(c, hipMemsetAsync(D.ntiles, 0, 2 * sizeof(int32_t), c->stream));
    HIPCHK(c, hipMemsetAsync(D.vmax_s, 0, sizeof(unsigned long long) * c->nbox * kStripes * kStripeStride, c->stream));
    HIPCHK(c, hipMemsetAsync(D.disp_s, 0, sizeof(unsigned long long) * c->nbox * kStripes * kStripeStride, c->stream));
    HIPCHK(c, hipHostMalloc((void**)&c->st_h, sizeof(BoxState) * c->nbox, hipHostMallocDefault));
    std::memset(c->st_h, 0, sizeof(BoxState) * c->nbox);
    for (int b = 0; b < c->nbox; ++b) c->st_h[b].vscale = 1.0;
    return MD_OK;
}

md_status check_ctx(md_ctx* c) {
    if (!c) return MD_EINVAL;
    if (c->sticky != MD_OK) return c->sticky;
    HIPCHK(c, hipSetDevice(c->device));
    return MD_OK;
}

// Copies the box states to the pinned mirror and waits.
md_status sync_states(md_ctx* c) {
    HIPCHK(c, hipMemcpyAsync(c->st_h, c->D.st, sizeof(BoxState) * c->nbox, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    LAUNCHCHK(c);
    if (c->timing) {
        for (size_t k = 0; k + 1 < c->ev_force.size(); k += 2) {
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, c->ev_force[k], c->ev_force[k + 1]));
            c->force_ms += ms;
            c->force_n += 1;
        }
        for (size_t k = 0; k + 1 < c->ev_rebuild.size(); k += 2) {
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, c->ev_rebuild[k], c->ev_rebuild[k + 1]));
            c->rebuild_ms += ms;
            c->rebuild_n += 1;
        }
    }
    for (hipEvent_t e : c->ev_force) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_rebuild) (void)hipEventDestroy(e);
    c->ev_force.clear();
    c->ev_rebuild.clear();
    return MD_OK;
}

// Uploads the pinned mirror of the box states (caller has synchronized).
md_status push_states(md_ctx* c) {
    HIPCHK(c, hipMemcpyAsync(c->D.st, c->st_h, sizeof(BoxState) * c->nbox, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MD_OK;
}

md_status timed_event(md_ctx* c, std::vector<hipEvent_t>& v) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreate(&e));
    HIPCHK(c, hipEventRecord(e, c->stream));
    v.push_back(e);
    return MD_OK;
}

md_status enqueue_rebuild(md_ctx* c, bool with_list) {
    md_status s;
    if (c->timing && (s = timed_event(c, c->ev_rebuild)) != MD_OK) return s;
    launch_rebuild_chain(c->D, c->P, with_list, c->stream);
    if (c->timing && (s = timed_event(c, c->ev_rebuild)) != MD_OK) return s;
    return MD_OK;
}

md_status enqueue_force(md_ctx* c, int mode, bool energy) {
    md_status s;
    if (c->timing && (s = timed_event(c, c->ev_force)) != MD_OK) return s;
    launch_force(c->D, c->P, mode, energy, c->stream);
    if (c->timing && (s = timed_event(c, c->ev_force)) != MD_OK) return s;
    if (c->prm.flags & MD_F_VERIFY_LIST) launch_verify(c->D, c->P, c->stream);
    return MD_OK;
}

// One continuing velocity-Verlet step: list rebuild chain (early exit unless
// flagged), forces with the closing and opening half kicks and the drift, DUTC.
md_status enqueue_mid_step(md_ctx* c) {
    md_status s;
    if ((s = enqueue_rebuild(c, true)) != MD_OK) return s;
    if ((s = enqueue_force(c, kForceMid, false)) != MD_OK) return s;
    launch_dutc(c->D, c->P, c->stream);
    return MD_OK;
}

md_status capture(md_ctx* c, int nsteps, hipGraphExec_t* out) {
    md_status s;
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < nsteps; ++k)
        if ((s = enqueue_mid_step(c)) != MD_OK) {
            (void)hipStreamEndCapture(c->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
    HIPCHK(c, hipStreamEndCapture(c->stream, &g));
    hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, MD_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return MD_OK;
}

// n continuing steps, as captured graphs when MD_F_GRAPH is set (and no
// per-kernel timing is requested), else kernel by kernel.
md_status enqueue_mid_steps(md_ctx* c, int n) {
    md_status s;
    const bool graphs = (c->prm.flags & MD_F_GRAPH) && !c->timing && c->stream != nullptr;
    if (!graphs) {
        for (int k = 0; k < n; ++k)
            if ((s = enqueue_mid_step(c)) != MD_OK) return s;
        return MD_OK;
    }
    if (!c->graph_many && (s = capture(c, kGraphSteps, &c->graph_many)) != MD_OK) return s;
    if (!c->graph_one && (s = capture(c, 1, &c->graph_one)) != MD_OK) return s;
    for (; n >= kGraphSteps; n -= kGraphSteps) HIPCHK(c, hipGraphLaunch(c->graph_many, c->stream));
    for (; n > 0; --n) HIPCHK(c, hipGraphLaunch(c->graph_one, c->stream));
    return MD_OK;
}

md_status status_from_states(md_ctx* c) {
    for (int b = 0; b < c->nbox; ++b) {
        if (c->st_h[b].err & 1)
            return fail(c, MD_ENUMERIC, "box %d: a position is not finite or lies outside [-L, 2L)", b);
        if (c->st_h[b].err & 2)
            return fail(c, MD_ENUMERIC, "box %d: a cell holds more than %d particles (overlapping particles?)", b,
                        kMaxCellCount);
    }
    return MD_OK;
}

int32_t max_need(const md_ctx* c) {
    int32_t m = 0;
    for (int b = 0; b < c->nbox; ++b) m = std::max(m, c->st_h[b].need);
    return m;
}

// Some box has a one-cell row tile whose staged region exceeds the capacity.
bool tile_overflow(const md_ctx* c) {
    for (int b = 0; b < c->nbox; ++b)
        if (c->st_h[b].err & 4) return true;
    return false;
}

// From now on the gather format: its lists need no staging capacity.  The caller
// has synchronized; the mirrored states lose the overflow bit.
md_status switch_to_gather(md_ctx* c) {
    c->tile_fallback = true;
    drop_graphs(c);
    params_refresh(c);
    for (int b = 0; b < c->nbox; ++b) c->st_h[b].err &= ~4;
    return MD_OK;
}


// Lets the kernels of a step run again after an overflow stopped them (a fill
// kernel, not a memset node, so the call is safe wherever it is enqueued).
void clear_halt(md_ctx* c) { launch_fill_i32(c->D.halt, 0, 1, c->stream); }

// Full list build for every box, growing the list until it fits.
md_status build_list(md_ctx* c) {
    md_status s;
    for (int attempt = 0; attempt < 8; ++attempt) {
        clear_halt(c);
        launch_mark_rebuild(c->D, c->P, c->stream);
        if ((s = enqueue_rebuild(c, true)) != MD_OK) return s;
        LAUNCHCHK(c);
        if ((s = sync_states(c)) != MD_OK) return s;
        if ((s = status_from_states(c)) != MD_OK) return s;
        if (tile_overflow(c)) {  // rebuild in the gather format
            switch_to_gather(c);
            for (int b = 0; b < c->nbox; ++b) c->st_h[b].need = 0;
            if ((s = push_states(c)) != MD_OK) return s;
            continue;
        }
        const int32_t need = max_need(c);
        if (need <= c->P.cap) {
            c->have_cells = c->have_list = true;
            c->have_F = false;
            return MD_OK;
        }
        // grow and rebuild (the overflow stopped the chain before the permuted buffers
        // became current; the rebuild sorts the same slots by cell again)
        if ((s = alloc_list(c, need + need / 4 + 8)) != MD_OK) return s;
        c->regrows += 1;
        for (int b = 0; b < c->nbox; ++b) c->st_h[b].need = 0;
        if ((s = push_states(c)) != MD_OK) return s;
    }
    return fail(c, MD_EHIP, "list capacity did not converge");
}

md_status ensure_list_and_forces(md_ctx* c) {
    md_status s;
    if (!c->have_state) return fail(c, MD_ESTATE, "no state: call md_set_state first");
    if (!c->have_list && (s = build_list(c)) != MD_OK) return s;
    if (!c->have_F) {
        if ((s = enqueue_force(c, kForceOnly, false)) != MD_OK) return s;
        LAUNCHCHK(c);
        c->have_F = true;
    }
    return MD_OK;
}

md_status reset_states_for_new_state(md_ctx* c, bool keep_series) {
    md_status s;
    clear_halt(c);
    if ((s = sync_states(c)) != MD_OK) return s;
    for (int b = 0; b < c->nbox; ++b) {
        BoxState& st = c->st_h[b];
        const int32_t ns = st.nseries, built = st.built;
        const unsigned long long missed = st.missed;
        const double thT = st.thT, thQ = st.thQ;  // the thermostat setting survives a new state
        std::memset(&st, 0, sizeof(BoxState));
        st.built = built;
        st.missed = missed;
        st.vscale = 1.0;
        st.thT = thT;
        st.thQ = thQ;
        if (keep_series) st.nseries = ns;
    }
    return push_states(c);
}

md_status create_impl(const md_params* boxes, int32_t nbox, void* stream, md_ctx** out) {
    if (!out) return MD_EINVAL;
    *out = nullptr;
    std::string why;
    md_status s = validate(boxes, nbox, why);
    g_create_err = why;
    if (s != MD_OK) return s;
    md_ctx* c = new (std::nothrow) md_ctx();
    if (!c) return MD_ENOMEM;
    c->nbox = nbox;
    c->prm = boxes[0];
    c->boxes.assign(boxes, boxes + nbox);
    hipError_t he = hipGetDevice(&c->device);
    if (he != hipSuccess) {
        g_create_err = std::string("hipGetDevice: ") + hipGetErrorString(he);
        delete c;
        return MD_EHIP;
    }
    // the fixed scratch of md_bubbles_noalloc: its device address on this device,
    // taken once per device while the device is current
    he = bubbles_scratch_init(c->device);
    if (he != hipSuccess) {
        g_create_err = std::string("hipGetSymbolAddress (bubble scratch): ") + hipGetErrorString(he);
        delete c;
        return MD_EHIP;
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        he = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (he != hipSuccess) {
            g_create_err = std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(he);
            delete c;
            return MD_EHIP;
        }
        c->own_stream = true;
    }
    layout(c);
    int tpk = c->prm.threads_per_key;
    // default layout (md_autotune measures instead): small systems need more lanes
    // per key to fill the chip; large ones are bound by partner gathers, where the
    // FP64 path's 32-byte records gain from two lanes reading adjacent entries
    if (tpk == 0) tpk = c->ntotal < 262144 ? 4 : (c->prm.precision == MD_PREC_FP64 ? 2 : 1);
    // Row tiles pay off on large boxes only: at 13.8M particles (FCC, density 0.5) their
    // force pass is 11% and the step 3.5% faster than the gather format's, at 4M particles
    // and below the gather format is 7-25% faster per step (the tile cuts cost rebuild time
    // and the gather pass's partners still hit in L2).  So the FP32-mixed default takes
    // them for a largest box of kTileMinN particles or more (md_autotune measures instead).
    int64_t nmax = 0;
    for (const md_params& bp : c->boxes) nmax = std::max(nmax, bp.n);
    const bool mixed = c->prm.precision == MD_PREC_FP32_MIXED;
    const bool tiles = !(c->prm.flags & (MD_F_TILE_OFF | MD_F_HALF_LIST)) &&
                       ((c->prm.flags & MD_F_TILE_ON) || (mixed && nmax >= kTileMinN));
    if (c->prm.threads_per_key == 0 && tiles) tpk = 1;
    c->prefer_gather = !tiles;
    if (c->prm.flags & MD_F_HALF_LIST) tpk = 1;
    c->P.tpk = tpk;
    params_refresh(c);
    if ((s = alloc_all(c)) != MD_OK || (s = upload_geometry(c)) != MD_OK ||
        (s = alloc_list(c, c->prm.list_cap > 0 ? c->prm.list_cap : estimate_cap(c))) != MD_OK) {
        g_create_err = c->err;
        free_all(c);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return s;
    }
    if ((s = push_states(c)) != MD_OK) {
        g_create_err = c->err;
        free_all(c);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return s;
    }
    *out = c;
    return MD_OK;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

md_status md_create(const md_params* params, void* stream, md_ctx** out) {
    return create_impl(params, 1, stream, out);
}

md_status md_batch_create(const md_params* boxes, int32_t nbox, void* stream, md_ctx** out) {
    return create_impl(boxes, nbox, stream, out);
}

md_status md_destroy(md_ctx* c) {
    if (!c) return MD_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return MD_OK;
}

md_status md_set_state(md_ctx* c, const double* pos, const double* vel) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!pos || !vel) return fail(c, MD_EINVAL, "pos and vel must be device pointers");
    if ((s = reset_states_for_new_state(c, false)) != MD_OK) return s;
    launch_set_state(c->D, c->P, pos, vel, c->nwave, c->stream);
    LAUNCHCHK(c);
    c->have_state = true;
    c->have_cells = c->have_list = c->have_F = false;
    return MD_OK;
}

md_status md_get_state(md_ctx* c, double* pos, double* vel) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!c->have_state) return fail(c, MD_ESTATE, "no state");
    launch_get_state(c->D, c->P, pos, vel, c->nwave, c->stream);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MD_OK;
}

md_status md_rescale_box(md_ctx* c, double alpha) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!c->have_state) return fail(c, MD_ESTATE, "no state");
    if (!finite_pos(alpha)) return fail(c, MD_EINVAL, "alpha must be finite and > 0");
    const double rl = c->prm.rc + c->prm.skin;
    for (int b = 0; b < c->nbox; ++b)
        for (int a = 0; a < 3; ++a) {
            const double L = c->boxes[b].box[a] * alpha;
            if (L < 3.0 * rl || std::floor(L / rl) > kMaxCellsPerAxis)
                return fail(c, MD_EINVAL, "box %d would leave the valid size range", b);
        }
    // scale positions first (kernel reads the current buffers), then the geometry
    std::vector<double> al(c->nbox, alpha);
    HIPCHK(c, hipMemcpyAsync(c->dscratch, al.data(), sizeof(double) * c->nbox, hipMemcpyHostToDevice, c->stream));
    launch_scale(c->D, c->P, c->dscratch, nullptr, c->stream);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < c->nbox; ++b)
        for (int a = 0; a < 3; ++a) c->boxes[b].box[a] *= alpha;
    c->prm.box[0] = c->boxes[0].box[0];
    c->prm.box[1] = c->boxes[0].box[1];
    c->prm.box[2] = c->boxes[0].box[2];
    layout(c);
    params_refresh(c);
    if ((s = alloc_cells(c)) != MD_OK) return s;
    if ((s = upload_geometry(c)) != MD_OK) return s;
    c->have_cells = c->have_list = c->have_F = false;
    return MD_OK;
}

md_status md_scale_velocities(md_ctx* c, const double* scale) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!c->have_state) return fail(c, MD_ESTATE, "no state");
    if (!scale) return fail(c, MD_EINVAL, "scale must be a host array [nbox]");
    for (int b = 0; b < c->nbox; ++b)
        if (!std::isfinite(scale[b])) return fail(c, MD_EINVAL, "scale factors must be finite");
    HIPCHK(c, hipMemcpyAsync(c->dscratch, scale, sizeof(double) * c->nbox, hipMemcpyHostToDevice, c->stream));
    launch_scale(c->D, c->P, nullptr, c->dscratch, c->stream);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MD_OK;
}

md_status md_build_cells(md_ctx* c) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!c->have_state) return fail(c, MD_ESTATE, "no state: call md_set_state first");
    for (int attempt = 0; attempt < 2; ++attempt) {
        clear_halt(c);
        launch_mark_rebuild(c->D, c->P, c->stream);
        if ((s = enqueue_rebuild(c, false)) != MD_OK) return s;
        LAUNCHCHK(c);
        if ((s = sync_states(c)) != MD_OK) return s;
        if ((s = status_from_states(c)) != MD_OK) return s;
        if (!tile_overflow(c)) break;
        // a row tile's staging capacity overflowed and stopped the chain: the
        // gather format from now on, and the cells again
        switch_to_gather(c);
        if ((s = push_states(c)) != MD_OK) return s;
    }
    c->have_cells = true;
    c->have_list = c->have_F = false;
    return MD_OK;
}

md_status md_build_neighbors(md_ctx* c) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!c->have_state) return fail(c, MD_ESTATE, "no state: call md_set_state first");
    return build_list(c);
}

md_status md_compute_forces(md_ctx* c, double* force) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!c->have_state) return fail(c, MD_ESTATE, "no state: call md_set_state first");
    if (!c->have_list && (s = build_list(c)) != MD_OK) return s;
    if ((s = enqueue_force(c, kForceOnly, false)) != MD_OK) return s;
    c->have_F = true;
    if (force) launch_get_forces(c->D, c->P, force, c->nwave, c->stream);
    LAUNCHCHK(c);
    if (c->prm.flags & MD_F_VERIFY_LIST) {
        if ((s = sync_states(c)) != MD_OK) return s;
        for (int b = 0; b < c->nbox; ++b)
            if (c->st_h[b].missed) return fail(c, MD_ELIST, "list verifier: pairs within rc missing from the list");
    }
    return MD_OK;
}

md_status md_step(md_ctx* c, int32_t nsteps, int32_t energy_every) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (nsteps < 0 || energy_every < 0) return fail(c, MD_EINVAL, "nsteps and energy_every must be >= 0");
    if ((s = ensure_list_and_forces(c)) != MD_OK) return s;
    if (nsteps == 0) return MD_OK;
    if ((s = sync_states(c)) != MD_OK) return s;
    bool thermo = false;
    for (int b = 0; b < c->nbox; ++b) thermo = thermo || c->st_h[b].thQ > 0.0;
    int32_t done = 0;
    // after an overflow: step done + 1 is already opened (kicked, drifted, DUTC checked)
    bool opened = false;
    while (done < nsteps) {
        const int32_t chunk = std::min(kChunk, nsteps - done);
        const int32_t nstep0 = c->st_h[0].nstep;
        for (int32_t k = 1; k <= chunk && thermo; ++k) {
            // Nose-Hoover: every step is kick/drift, forces with the closing kick and the
            // energy partials, then the thermostat half steps (end of this step and start
            // of the next) folded into the next kick; the run ends with the velocities
            // scaled by the closing half step's factor
            const int32_t gk = done + k;
            if (k == 1 && !opened) {
                launch_ke_partial(c->D, c->P, c->stream);
                launch_energy_reduce(c->D, c->P, false, 2, false, c->stream);
                launch_kick_drift(c->D, c->P, c->stream);
                launch_dutc(c->D, c->P, c->stream);
            }
            const bool energy = energy_every > 0 && gk % energy_every == 0;
            const bool last = k == chunk;
            if ((s = enqueue_rebuild(c, true)) != MD_OK) return s;
            if ((s = enqueue_force(c, kForceEnd, true)) != MD_OK) return s;
            launch_energy_reduce(c->D, c->P, energy, last ? 1 : 3, c->P.tile != 0, c->stream);
            if (last) {
                launch_vscale(c->D, c->P, c->stream);
            } else {
                launch_kick_drift(c->D, c->P, c->stream);
                launch_dutc(c->D, c->P, c->stream);
            }
        }
        for (int32_t k = 1; k <= chunk && !thermo; ++k) {
            const int32_t gk = done + k;
            if (k == 1 && !opened) {
                launch_kick_drift(c->D, c->P, c->stream);
                launch_dutc(c->D, c->P, c->stream);
            }
            const bool energy = energy_every > 0 && gk % energy_every == 0;
            const bool last = k == chunk;
            if (energy || last) {
                if ((s = enqueue_rebuild(c, true)) != MD_OK) return s;
                if ((s = enqueue_force(c, kForceEnd, energy)) != MD_OK) return s;
                if (energy) launch_energy_reduce(c->D, c->P, true, 0, c->P.tile != 0, c->stream);
                if (!last) {
                    launch_kick_drift(c->D, c->P, c->stream);
                    launch_dutc(c->D, c->P, c->stream);
                }
            } else {
                // a run of continuing steps up to the next energy sample or chunk end
                int32_t run = 1;
                while (k + run < chunk && !(energy_every > 0 && (gk + run) % energy_every == 0)) ++run;
                if ((s = enqueue_mid_steps(c, run)) != MD_OK) return s;
                k += run - 1;
            }
        }
        LAUNCHCHK(c);
        if ((s = sync_states(c)) != MD_OK) return s;
        if ((s = status_from_states(c)) != MD_OK) return s;
        const int32_t need = max_need(c);
        const bool tover = tile_overflow(c);
        if (need > c->P.cap || tover) {
            // A list build overflowed (list capacity, or a row tile's staging capacity)
            // and every kernel after it returned at once: the state is the one that
            // build found, in step `open` of this chunk (kicked, drifted, DUTC checked,
            // list pending).  Grow the list or change its format and go on from there.
            const int32_t open = (opened ? 1 : 0) + (c->st_h[0].nstep - nstep0);
            clear_halt(c);
            if (need > c->P.cap) {
                if ((s = grow_list_keeping(c, need + need / 4 + 8)) != MD_OK) {
                    c->have_list = c->have_F = false;  // the state is step `open`, drifted
                    return s;
                }
                c->regrows += 1;
            }
            if (tover) {
                // the gather format reads no row-tile entries: every box builds again
                switch_to_gather(c);
                for (int b = 0; b < c->nbox; ++b) c->st_h[b].rebuild = 1;
            }
            if ((s = push_states(c)) != MD_OK) return s;
            if (tover) launch_mark_rebuild(c->D, c->P, c->stream);
            done += open - 1;
            c->steps += open - 1;
            opened = true;
            continue;
        }
        if (thermo) {  // k_vscale applied the pending factor: the next kick starts from 1
            for (int b = 0; b < c->nbox; ++b) c->st_h[b].vscale = 1.0;
            if ((s = push_states(c)) != MD_OK) return s;
        }
        done += chunk;
        c->steps += chunk;
        opened = false;
    }
    c->have_F = true;
    if (c->prm.flags & MD_F_VERIFY_LIST)
        for (int b = 0; b < c->nbox; ++b)
            if (c->st_h[b].missed) return fail(c, MD_ELIST, "list verifier: pairs within rc missing from the list");
    return MD_OK;
}

static md_status energies(md_ctx* c) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!c->have_state) return fail(c, MD_ESTATE, "no state: call md_set_state first");
    if (!c->have_list && (s = build_list(c)) != MD_OK) return s;
    if ((s = enqueue_force(c, kForceOnly, true)) != MD_OK) return s;
    c->have_F = true;
    launch_energy_reduce(c->D, c->P, false, 0, c->P.tile != 0, c->stream);
    LAUNCHCHK(c);
    return sync_states(c);
}

md_status md_energy(md_ctx* c, double* ke, double* pe) {
    md_status s = energies(c);
    if (s != MD_OK) return s;
    double k = 0.0, e = 0.0;
    for (int b = 0; b < c->nbox; ++b) {
        k += c->st_h[b].ke;
        e += c->st_h[b].pe;
    }
    if (ke) *ke = k;
    if (pe) *pe = e;
    return MD_OK;
}

md_status md_batch_energy(md_ctx* c, double* ke, double* pe) {
    md_status s = energies(c);
    if (s != MD_OK) return s;
    for (int b = 0; b < c->nbox; ++b) {
        if (ke) ke[b] = c->st_h[b].ke;
        if (pe) pe[b] = c->st_h[b].pe;
    }
    return MD_OK;
}

md_status md_energy_series(md_ctx* c, double* ke, double* pe, int32_t max, int32_t* count) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if ((s = sync_states(c)) != MD_OK) return s;
    int32_t n = c->st_h[0].nseries;
    if (count) *count = n;
    n = std::min(n, std::max(max, 0));
    if (n > 0 && ke)
        HIPCHK(c, hipMemcpy(ke, c->D.series_ke, sizeof(double) * n * c->nbox, hipMemcpyDeviceToHost));
    if (n > 0 && pe)
        HIPCHK(c, hipMemcpy(pe, c->D.series_pe, sizeof(double) * n * c->nbox, hipMemcpyDeviceToHost));
    return MD_OK;
}

md_status md_observable_series(md_ctx* c, double* vir, double* thermostat, int32_t max, int32_t* count) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if ((s = sync_states(c)) != MD_OK) return s;
    int32_t n = c->st_h[0].nseries;
    if (count) *count = n;
    n = std::min(n, std::max(max, 0));
    if (n > 0 && vir)
        HIPCHK(c, hipMemcpy(vir, c->D.series_vir, sizeof(double) * n * c->nbox, hipMemcpyDeviceToHost));
    if (n > 0 && thermostat)
        HIPCHK(c, hipMemcpy(thermostat, c->D.series_th, sizeof(double) * n * c->nbox, hipMemcpyDeviceToHost));
    return MD_OK;
}

md_status md_pressure(md_ctx* c, double* pressure) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!pressure) return fail(c, MD_EINVAL, "pressure must not be NULL");
    if ((s = energies(c)) != MD_OK) return s;
    for (int b = 0; b < c->nbox; ++b) {
        const double V = c->boxes[b].box[0] * c->boxes[b].box[1] * c->boxes[b].box[2];
        pressure[b] = (2.0 * c->st_h[b].ke - c->st_h[b].vir) / (3.0 * V);
    }
    return MD_OK;
}

md_status md_set_thermostat(md_ctx* c, const double* T, double tau) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!std::isfinite(tau)) return fail(c, MD_EINVAL, "tau must be finite");
    if (tau > 0.0) {
        if (!T) return fail(c, MD_EINVAL, "T must not be NULL when tau > 0");
        for (int b = 0; b < c->nbox; ++b)
            if (!(T[b] > 0.0) || !std::isfinite(T[b])) return fail(c, MD_EINVAL, "T[%d] must be > 0", b);
    }
    if ((s = sync_states(c)) != MD_OK) return s;
    for (int b = 0; b < c->nbox; ++b) {
        BoxState& st = c->st_h[b];
        const double g = 3.0 * (double)c->boxes[b].n - 3.0;
        st.thT = tau > 0.0 ? T[b] : 0.0;
        st.thQ = tau > 0.0 ? g * T[b] * tau * tau : 0.0;
        st.xi = st.eta = 0.0;
        st.vscale = 1.0;
    }
    return push_states(c);
}

md_status md_bubbles(md_ctx* c, int32_t box, double side, double rho_gas, uint8_t* counts, int32_t* labels,
                     int64_t* roots, int64_t* sizes, int64_t cap, md_bubble_info* info) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!info) return fail(c, MD_EINVAL, "info must not be NULL");
    if (box < 0 || box >= c->nbox) return fail(c, MD_EINVAL, "box %d out of range [0, %d)", box, c->nbox);
    if (!finite_pos(side)) return fail(c, MD_EINVAL, "side must be finite and > 0");
    if (!(rho_gas >= 0.0) || !std::isfinite(rho_gas)) return fail(c, MD_EINVAL, "rho_gas must be finite and >= 0");
    if (cap < 0 || (cap > 0 && (!roots || !sizes))) return fail(c, MD_EINVAL, "roots and sizes need cap entries");
    if (!c->have_state) return fail(c, MD_ESTATE, "no state: call md_set_state first");
    SubGrid sg{};
    const double* L = c->boxes[box].box;
    for (int a = 0; a < 3; ++a) {
        const double n = std::floor(L[a] / side);
        if (n < 1.0 || n > 1024.0)
            return fail(c, MD_EINVAL, "floor(L / side) = %.0f on axis %d: need 1..1024 subcells", n, a);
        sg.L[a] = L[a];
        sg.n[a] = (int32_t)n;
        sg.inv[a] = (double)sg.n[a] / L[a];
    }
    const double vol = (L[0] / sg.n[0]) * (L[1] / sg.n[1]) * (L[2] / sg.n[2]);
    sg.thr = rho_gas * vol;
    const int64_t nsub = (int64_t)sg.n[0] * sg.n[1] * sg.n[2];
    sg.nsub = (int32_t)nsub;
    if (nsub > c->bw_alloc) {
        dfree(c->bw.cnt);
        dfree(c->bw.par);
        dfree(c->bw.lab);
        dfree(c->bw.size);
        dfree(c->bw.roots);
        dfree(c->bw.flag);
        c->bw_alloc = 0;
        if ((s = dalloc(c, &c->bw.cnt, nsub)) != MD_OK || (s = dalloc(c, &c->bw.par, nsub)) != MD_OK ||
            (s = dalloc(c, &c->bw.lab, nsub)) != MD_OK || (s = dalloc(c, &c->bw.size, nsub)) != MD_OK ||
            (s = dalloc(c, &c->bw.roots, nsub)) != MD_OK || (s = dalloc(c, &c->bw.flag, 2)) != MD_OK)
            return s;
        c->bw_alloc = nsub;
    }
    HIPCHK(c, hipMemsetAsync(c->bw.cnt, 0, sizeof(uint32_t) * nsub, c->stream));
    HIPCHK(c, hipMemsetAsync(c->bw.flag, 0, sizeof(int32_t) * 2, c->stream));
    launch_bubbles(c->D, box, c->geom[box].npart, sg, c->bw, counts, c->stream);
    LAUNCHCHK(c);
    if (labels)
        HIPCHK(c, hipMemcpyAsync(labels, c->bw.lab, sizeof(int32_t) * nsub, hipMemcpyDeviceToDevice, c->stream));
    int32_t flag[2] = {0, 0};
    HIPCHK(c, hipMemcpyAsync(flag, c->bw.flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flag[0]) return fail(c, MD_ENUMERIC, "box %d: a position is not finite or lies outside [-L, 2L)", box);
    std::vector<int2> rs((size_t)flag[1]);
    if (flag[1] > 0) {
        HIPCHK(c, hipMemcpy(rs.data(), c->bw.roots, sizeof(int2) * rs.size(), hipMemcpyDeviceToHost));
        std::sort(rs.begin(), rs.end(), [](const int2& a, const int2& b) { return a.x < b.x; });
    }
    int64_t ngas = 0, largest = 0;
    for (const int2& r : rs) {
        ngas += r.y;
        largest = std::max<int64_t>(largest, r.y);
    }
    for (int64_t k = 0; k < cap && k < (int64_t)rs.size(); ++k) {
        roots[k] = rs[k].x;
        sizes[k] = rs[k].y;
    }
    *info = md_bubble_info{};
    for (int a = 0; a < 3; ++a) {
        info->nsub[a] = sg.n[a];
        info->side[a] = L[a] / sg.n[a];
    }
    info->threshold = sg.thr;
    info->ngas = ngas;
    info->nbubbles = (int64_t)rs.size();
    info->largest = largest;
    return MD_OK;
}

md_status md_bubbles_noalloc(md_ctx* c, int32_t box, double side, double rho_gas, uint8_t* counts, int32_t* labels,
                             int64_t* roots, int64_t* sizes, int64_t cap, md_bubble_info* info) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!info) return fail(c, MD_EINVAL, "info must not be NULL");
    if (box < 0 || box >= c->nbox) return fail(c, MD_EINVAL, "box %d out of range [0, %d)", box, c->nbox);
    if (!finite_pos(side)) return fail(c, MD_EINVAL, "side must be finite and > 0");
    if (!(rho_gas >= 0.0) || !std::isfinite(rho_gas)) return fail(c, MD_EINVAL, "rho_gas must be finite and >= 0");
    if (cap < 0 || (cap > 0 && (!roots || !sizes))) return fail(c, MD_EINVAL, "roots and sizes need cap entries");
    if (!c->have_state) return fail(c, MD_ESTATE, "no state: call md_set_state first");
    unsigned char* base = bubbles_scratch(c->device);
    if (!base) return fail(c, MD_EHIP, "no fixed bubble scratch on device %d", c->device);
    SubGrid sg{};
    const double* L = c->boxes[box].box;
    int64_t nsub = 1;
    for (int a = 0; a < 3; ++a) {
        const double n = std::floor(L[a] / side);
        if (n < 1.0 || n > 1024.0)
            return fail(c, MD_EINVAL, "floor(L / side) = %.0f on axis %d: need 1..1024 subcells", n, a);
        sg.L[a] = L[a];
        sg.n[a] = (int32_t)n;
        sg.inv[a] = (double)sg.n[a] / L[a];
        nsub *= sg.n[a];
    }
    if (nsub > kNaMaxSub)
        return fail(c, MD_EINVAL, "%lld subcells exceed the fixed scratch of md_bubbles_noalloc (%d subcells)",
                    (long long)nsub, kNaMaxSub);
    const double vol = (L[0] / sg.n[0]) * (L[1] / sg.n[1]) * (L[2] / sg.n[2]);
    sg.thr = rho_gas * vol;
    sg.nsub = (int32_t)nsub;
    launch_bubbles_scratch(c->D, box, c->geom[box].npart, sg, base, counts, c->stream);
    LAUNCHCHK(c);
    int64_t *d_root, *d_rsize;
    int32_t* d_lab;
    NaMisc* d_misc;
    bubbles_scratch_results(base, &d_root, &d_rsize, &d_lab, &d_misc);
    if (labels)
        HIPCHK(c, hipMemcpyAsync(labels, d_lab, sizeof(int32_t) * nsub, hipMemcpyDeviceToDevice, c->stream));
    NaMisc m{};
    HIPCHK(c, hipMemcpyAsync(&m, d_misc, sizeof m, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (m.bad) return fail(c, MD_ENUMERIC, "box %d: a position is not finite or lies outside [-L, 2L)", box);
    const int64_t k = std::min<int64_t>(cap, m.nroots);
    if (k > 0) {
        HIPCHK(c, hipMemcpyAsync(roots, d_root, sizeof(int64_t) * k, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(sizes, d_rsize, sizeof(int64_t) * k, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    *info = md_bubble_info{};
    for (int a = 0; a < 3; ++a) {
        info->nsub[a] = sg.n[a];
        info->side[a] = L[a] / sg.n[a];
    }
    info->threshold = sg.thr;
    info->ngas = (int64_t)m.ngas;
    info->nbubbles = m.nroots;
    info->largest = m.largest;
    return MD_OK;
}

md_status md_get_thermostat(md_ctx* c, double* xi, double* eta) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if ((s = sync_states(c)) != MD_OK) return s;
    for (int b = 0; b < c->nbox; ++b) {
        if (xi) xi[b] = c->st_h[b].xi;
        if (eta) eta[b] = c->st_h[b].eta;
    }
    return MD_OK;
}

md_status md_get_cells(md_ctx* c, int32_t* cell_of_particle, int32_t* ncell) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!c->have_cells) return fail(c, MD_ESTATE, "no binning since the last state change");
    if (ncell) {
        ncell[0] = c->geom[0].n[0];
        ncell[1] = c->geom[0].n[1];
        ncell[2] = c->geom[0].n[2];
    }
    if (cell_of_particle) launch_get_cells(c->D, c->P, cell_of_particle, c->nwave, c->stream);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MD_OK;
}

md_status md_get_neighbors(md_ctx* c, int64_t* key_ptr, int32_t* partners, int64_t cap, int64_t* total) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!c->have_list) return fail(c, MD_ESTATE, "no valid pair list");
    if (!key_ptr) return fail(c, MD_EINVAL, "key_ptr must be a device array [n + 1]");
    launch_list_counts(c->D, c->P, key_ptr + 1, c->nwave, c->stream);
    LAUNCHCHK(c);
    std::vector<int64_t> kp(c->ntotal + 1, 0);
    HIPCHK(c, hipMemcpyAsync(kp.data() + 1, key_ptr + 1, sizeof(int64_t) * c->ntotal, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < c->ntotal; ++i) kp[i + 1] += kp[i];
    HIPCHK(c, hipMemcpy(key_ptr, kp.data(), sizeof(int64_t) * kp.size(), hipMemcpyHostToDevice));
    if (total) *total = kp[c->ntotal];
    if (kp[c->ntotal] > cap) return fail(c, MD_EINVAL, "partners capacity %lld < %lld entries", (long long)cap,
                                         (long long)kp[c->ntotal]);
    if (!partners) return fail(c, MD_EINVAL, "partners must be a device array");
    launch_list_export(c->D, c->P, key_ptr, partners, c->nwave, c->stream);
    LAUNCHCHK(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return MD_OK;
}

md_status md_get_stats(md_ctx* c, md_stats* out) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if (!out) return fail(c, MD_EINVAL, "null stats pointer");
    if ((s = sync_states(c)) != MD_OK) return s;
    std::memset(out, 0, sizeof(*out));
    out->steps = c->steps;
    out->list_regrows = c->regrows;
    int32_t mx = 0;
    for (int b = 0; b < c->nbox; ++b) {
        out->rebuilds += c->st_h[b].built;
        out->missed_pairs += (int64_t)c->st_h[b].missed;
        mx = std::max(mx, c->st_h[b].need);
    }
    out->max_list_len = mx;
    out->list_cap = c->P.cap;
    out->threads_per_key = c->P.tpk;
    out->nbox = c->nbox;
    out->D = c->st_h[0].D;
    out->force_ms = c->force_ms;
    out->force_launches = c->force_n;
    out->rebuild_ms = c->rebuild_ms;
    out->rebuild_launches = c->rebuild_n;
    out->row_tiles = c->P.tile;
    for (int a = 0; a < 3; ++a) out->ncell[a] = c->geom[0].n[a];
    out->cell_scale = cell_scale_of(c);
    if (c->have_list) {
        std::vector<int32_t> cnt(c->nslot);
        HIPCHK(c, hipMemcpy(cnt.data(), c->D.cnt, sizeof(int32_t) * c->nslot, hipMemcpyDeviceToHost));
        int64_t tot = 0;
        for (int b = 0; b < c->nbox; ++b) {
            const BoxGeom& g = c->geom[b];
            for (int k = 0; k < g.npart; ++k) tot += cnt[g.slot_off + k];
        }
        out->list_entries = tot;
    }
    return MD_OK;
}

md_status md_set_timing(md_ctx* c, int32_t on) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if ((s = sync_states(c)) != MD_OK) return s;
    c->timing = on != 0;
    c->force_ms = c->rebuild_ms = 0.0;
    c->force_n = c->rebuild_n = 0;
    return MD_OK;
}

md_status md_autotune(md_ctx* c, const char* cache_path) {
    md_status s;
    if ((s = check_ctx(c)) != MD_OK) return s;
    if ((s = ensure_list_and_forces(c)) != MD_OK) return s;
    if (c->P.half) return MD_OK;  // a half list has one layout: one lane per key
    // cache key: precision, density (1/20 steps), particles per box (log2), ensemble or not
    double rho = 0.0, nmean = 0.0;
    for (int b = 0; b < c->nbox; ++b) {
        const md_params& p = c->boxes[b];
        rho += (double)p.n / (p.box[0] * p.box[1] * p.box[2]) / c->nbox;
        nmean += (double)p.n / c->nbox;
    }
    char key[96];
    snprintf(key, sizeof key, "%d %d %d %d", c->prm.precision, (int)std::lround(rho * 20.0),
             (int)std::lround(std::log2(nmean)), c->nbox > 1 ? 1 : 0);

    // candidates the parameters allow
    struct Cand {
        int tpk;
        bool tile;
        int pct;  // cell_scale in percent
    };
    const uint32_t fl = c->prm.flags;
    std::vector<int> pcts;
    if (c->prm.cell_scale > 0.0)
        pcts.push_back((int)std::lround(c->prm.cell_scale * 100.0));
    else
        pcts = {100, 115, 130};
    std::vector<Cand> cands;
    for (int pct : pcts) {
        if (!(fl & MD_F_TILE_OFF) && (c->prm.threads_per_key == 0 || c->prm.threads_per_key == 1))
            cands.push_back({1, true, pct});
        if (fl & MD_F_TILE_ON) continue;
        for (int t : {1, 2, 4, 8})
            if (c->prm.threads_per_key == 0 || c->prm.threads_per_key == t) cands.push_back({t, false, pct});
    }
    auto valid = [&](const Cand& k) {
        for (const Cand& q : cands)
            if (q.tpk == k.tpk && q.tile == k.tile && q.pct == k.pct) return true;
        return false;
    };

    Cand best{0, false, 0};
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            if (line.empty() || line[0] == '#') continue;
            std::istringstream ls(line);
            int a, b2, c2, d2, t, tl, pct;
            if (ls >> a >> b2 >> c2 >> d2 >> t >> tl >> pct) {
                char k2[96];
                snprintf(k2, sizeof k2, "%d %d %d %d", a, b2, c2, d2);
                const Cand k{t, tl != 0, pct};
                if (std::strcmp(k2, key) == 0 && valid(k)) best = k;
            }
        }
    }
    if (!c->bk_pos && (s = dalloc(c, &c->bk_pos, (size_t)c->ntotal * 3)) != MD_OK) return s;
    if (!c->bk_vel && (s = dalloc(c, &c->bk_vel, (size_t)c->ntotal * 3)) != MD_OK) return s;
    // the state's own rebuild counts are kept; the builds made here are not steps
    if ((s = sync_states(c)) != MD_OK) return s;
    std::vector<int32_t> built(c->nbox);
    for (int b = 0; b < c->nbox; ++b) built[b] = c->st_h[b].built;
    const double interval = c->steps > 0 && built[0] > 0 ? (double)c->steps / built[0] : 10.0;
    const bool fallback0 = c->tile_fallback;

    // re-lay the grid and the list for candidate k and build the list.  The slots go
    // back to caller order first (as md_set_state leaves them), so that the order
    // within cells after the last build does not depend on the candidates timed
    // before it: a tuned context and one that reads the choice from the cache step
    // identically.
    auto apply = [&](const Cand& k) -> md_status {
        md_status r;
        if ((r = sync_states(c)) != MD_OK) return r;
        launch_get_state(c->D, c->P, c->bk_pos, c->bk_vel, c->nwave, c->stream);
        for (int b = 0; b < c->nbox; ++b) {
            BoxState& st = c->st_h[b];
            st.sq = st.sp = 0;
            st.need = 0;
            st.rebuild = 0;
        }
        if ((r = push_states(c)) != MD_OK) return r;
        launch_set_state(c->D, c->P, c->bk_pos, c->bk_vel, c->nwave, c->stream);
        LAUNCHCHK(c);
        c->cell_scale = k.pct / 100.0;
        c->prefer_gather = !k.tile;
        c->tile_fallback = fallback0;
        c->P.tpk = k.tpk;
        layout(c);
        params_refresh(c);
        if ((r = alloc_cells(c)) != MD_OK) return r;
        if ((r = upload_geometry(c)) != MD_OK) return r;
        if ((r = alloc_list(c, c->P.cap)) != MD_OK) return r;
        c->have_cells = c->have_list = c->have_F = false;
        return build_list(c);
    };

    const bool from_cache = best.tpk != 0;
    if (!from_cache) {
        float best_cost = 1e30f;
        hipEvent_t ev[3];
        for (hipEvent_t& e : ev) HIPCHK(c, hipEventCreate(&e));
        for (const Cand& k : cands) {
            if ((s = apply(k)) != MD_OK) return s;
            if (k.tile && !c->P.tile) continue;  // the tiles overflowed: a gather candidate covers it
            // the chain again on sorted slots (re-sorts identically), then forces
            HIPCHK(c, hipEventRecord(ev[0], c->stream));
            launch_mark_rebuild(c->D, c->P, c->stream);
            launch_rebuild_chain(c->D, c->P, true, c->stream);
            HIPCHK(c, hipEventRecord(ev[1], c->stream));
            launch_force(c->D, c->P, kForceOnly, false, c->stream);  // warm-up
            for (int r = 0; r < 5; ++r) launch_force(c->D, c->P, kForceOnly, false, c->stream);
            HIPCHK(c, hipEventRecord(ev[2], c->stream));
            HIPCHK(c, hipEventSynchronize(ev[2]));
            LAUNCHCHK(c);
            float mr = 0.f, mf = 0.f;
            HIPCHK(c, hipEventElapsedTime(&mr, ev[0], ev[1]));
            HIPCHK(c, hipEventElapsedTime(&mf, ev[1], ev[2]));
            const float cost = mf / 6.0f + mr / (float)interval;
            if (cost < best_cost) {
                best_cost = cost;
                best = k;
            }
        }
        for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
    }
    if ((s = apply(best)) != MD_OK) return s;
    if ((s = ensure_list_and_forces(c)) != MD_OK) return s;
    if ((s = sync_states(c)) != MD_OK) return s;
    for (int b = 0; b < c->nbox; ++b) c->st_h[b].built = built[b];
    if ((s = push_states(c)) != MD_OK) return s;
    if (cache_path && !from_cache) {
        std::ofstream out(cache_path, std::ios::app);
        if (out) out << key << " " << best.tpk << " " << (best.tile ? 1 : 0) << " " << best.pct << "\n";
    }
    return MD_OK;
}

const char* md_status_str(md_status s) {
    // a C caller may pass any int; its bits are read as an int, since reading an
    // out-of-range value through the C++ enum type is undefined
    int v;
    std::memcpy(&v, &s, sizeof v);
    const int k = -v;
    if (k < 0 || k >= (int)(sizeof(kStatusStr) / sizeof(kStatusStr[0]))) return "MD_UNKNOWN";
    return kStatusStr[k];
}

const char* md_last_error(const md_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

}  // extern "C"
