// md_kernels.hip -- gfx950 kernels of the short-range LJ hot path.
//
// Per step (velocity Verlet, Sec. III.B; list validity by DUTC, Sec. II.A):
//   force pass (kForceMid)  close step n (v += hF), open step n+1 (v += hF, q += dt v),
//                           per-box max |v|^2 for the DUTC bound: k_force_t (FP32-mixed,
//                           partners from a row tile staged in LDS) or k_force (gather
//                           format: FP64, and FP32-mixed when tiles do not fit)
//   k_dutc                  D += dt * max|v|; flag a rebuild when 2D > skin
//   rebuild chain           (early exit unless flagged) wrap + cell id, counting sort
//                           by cell, permute into coalesced arrays, row tiles, pair list
// and at chunk ends the force pass in kForceEnd mode (closing half kick, F stored)
// followed by k_kick_drift at the start of the next chunk.
//
// The force passes follow Algorithm 1 (Sec. III.C): a full list, each key's force
// summed by its own lane(s) and never scattered, the momentum update fused into
// the force pass.  The truncation mask of Algorithm 1 becomes a select, or for the
// Eq. (1) cutoff on the FP32-mixed passes a clamp of 1/r^2 at 1/rc^2 (f(rc) = 0);
// no lane branches on it.  Parallel work is one lane (or tpk lanes) per key over a
// wave-blocked ELL list, so list reads are coalesced.
#include <math.h>

#include <type_traits>

#include "md.h"
#include "md_internal.h"

namespace mdg {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Index of the calling wavefront within its block, in a scalar register.
__device__ __forceinline__ int wave_in_block() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Streaming accesses of the force pass (list chunks, velocities): each byte is used
// once per pass, so they carry the non-temporal hint and leave the L2 to the partner
// records that neighbouring wavefronts gather again.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
    const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }

// A wave-uniform read of a value the running kernel does not write, through the
// constant address space, so it becomes a scalar load (scalar cache).
__device__ __forceinline__ int ld_const(const int32_t* p) {
    return *reinterpret_cast<const __attribute__((address_space(4))) int32_t*>(
        reinterpret_cast<uintptr_t>(p));
}

// A list build of this step overflowed (the list's capacity, or a row tile's
// staging capacity): every kernel of a step returns at once, leaving the state as
// that build found it, until the host has grown the list or changed its format.
__device__ __forceinline__ bool halted(const Dev& d) { return ld_const(d.halt) != 0; }

// A box's geometry, read through the scalar cache: no kernel writes it, so the
// wavefront-uniform reads become scalar loads instead of a chain of vector loads
// that every store in a loop would force to repeat.
__device__ __forceinline__ BoxGeom ld_geom(const BoxGeom* p) {
    static_assert(sizeof(BoxGeom) % 4 == 0, "BoxGeom is copied as 32-bit words");
    const __attribute__((address_space(4))) int32_t* src =
        reinterpret_cast<const __attribute__((address_space(4))) int32_t*>(reinterpret_cast<uintptr_t>(p));
    BoxGeom g;
    int32_t* dst = reinterpret_cast<int32_t*>(&g);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(BoxGeom) / 4); ++i) dst[i] = src[i];  // unused words are never loaded
    return g;
}

// x / n[0] (k = 0), x / n[1] (k = 1) or x / (n[0] * n[1]) (k = 2) for 0 <= x < 2^30,
// with the box's precomputed multiplier and shift instead of an integer division.
__device__ __forceinline__ int gdiv(const BoxGeom& g, int x, int k) {
    return (int)(__umulhi((uint32_t)x, g.dmul[k]) >> g.dshr[k]);
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Give XCD x a contiguous run of logical blocks so that neighbouring
// keys, whose partners overlap, share that XCD's L2.  Bijective on [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int l = lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o);
        if (l >= o) v += t;
    }
    return v;
}

// Inclusive running maximum over the 64 lanes of non-negative values, by DPP lane
// moves: shifts by 1, 2, 4, 8 within each row of 16 lanes, then the last lane of
// each row broadcast into the rows after it.  A lane whose source is outside its
// row, or whose row the mask leaves out, receives 0, the identity.  Every lane
// must be active.
__device__ __forceinline__ int wave_incl_max(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));  // row_bcast:15 into rows 1, 3
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));  // row_bcast:31 into rows 2, 3
    return v;
}

// Inclusive sum over the 64 lanes by the same DPP lane moves (0 is the identity).
// Every lane must be active.
__device__ __forceinline__ int wave_incl_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return v;
}

// Exclusive scan across a 256-thread block; *total gets the block sum.
__device__ int block_excl_scan(int v, int* total) {
    __shared__ int ws[kBlock / kWave];
    const int wib = threadIdx.x >> 6, l = lane_id();
    int inc = wave_incl_scan(v);
    if (l == 63) ws[wib] = inc;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
        if (w < wib) off += ws[w];
        tot += ws[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Fixed-point cell-relative coordinate of x in cell c (2^28 units per cell side,
// relative to the cell centre (c + 1/2) * cs), clamped to two cell sides so pair
// differences never overflow int32.
// No contraction: every kernel that encodes a position (binning permutation, drifts,
// the force passes' own coordinate) must round the anchor product, the difference and
// the scaling alike, or a particle's record could differ by one unit between them.
__device__ __forceinline__ int to_units(double x, int c, double cs, double ucs) {
#pragma clang fp contract(off)
    const double a = ((double)c + 0.5) * cs;  // the anchor
    double t = rint((x - a) * ucs);
    t = fmin(fmax(t, -(double)kUnitClamp), (double)kUnitClamp);
    return (int)t;
}

__device__ __forceinline__ Pos make_pos(double x, double y, double z, uint32_t cc, int32_t cnt) {
    Pos r;
    r.x = x;
    r.y = y;
    r.z = z;
    r.cc = cc;
    r.cnt = cnt;
    return r;
}

// Global fixed-point coordinate of x, modulo 2^32: c * uoff + the cell-relative
// units, c = the particle's cell at the last build.  Any two particles' difference
// (plus a periodic image term n * uoff) is their exact separation in units, since
// it stays far inside int32; a block can therefore stage any run of cells with a
// plain copy.
__device__ __forceinline__ int gunit(double x, int c, double cs, double ucs, int32_t uoff) {
    return (int)((uint32_t)to_units(x, c, cs, ucs) + (uint32_t)c * (uint32_t)uoff);
}
__device__ __forceinline__ int4 units3(const Pos& x, uint32_t cc, const BoxGeom& g) {
    return make_int4(gunit(x.x, cc & 1023, g.cs[0], g.ucs, g.uoff[0]),
                     gunit(x.y, (cc >> 10) & 1023, g.cs[1], g.ucs, g.uoff[1]),
                     gunit(x.z, cc >> 20, g.cs[2], g.ucs, g.uoff[2]), 0);
}
// The image term of a periodic image r (r = +1 where the partner's cell index wrapped
// below 0), per axis, modulo 2^32: -r * n * uoff.
__device__ __forceinline__ int img_units(int r, int n, int32_t uoff) {
    return (int)(uint32_t)(-(int64_t)r * (int64_t)n * (int64_t)uoff);
}


// Fixed-point position record of the FP32-mixed path: 12 bytes, 4-byte aligned,
// so records pack densely and a gather of one record is one dwordx3 load.
struct __attribute__((packed, aligned(4))) U3 {
    int x, y, z;
};
__device__ __forceinline__ void put_u(int32_t* u, int s, int4 v) { *reinterpret_cast<U3*>(u + 3 * s) = U3{v.x, v.y, v.z}; }
__device__ __forceinline__ int4 get_u(const int32_t* u, int s) {
    const U3 t = *reinterpret_cast<const U3*>(u + 3 * s);
    return make_int4(t.x, t.y, t.z, 0);
}

// ---------------------------------------------------------------- state I/O

__global__ __launch_bounds__(kBlock) void k_set_state(Dev d, Params p, const double* __restrict__ pos,
                                                      const double* __restrict__ vel) {
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        const int k = s - g.slot_off;
        if (k >= g.npart) continue;
        const int64_t i = (int64_t)g.id_off + k;
        d.q[0][s] = make_pos(pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], 0u, 0);
        d.vx[0][s] = vel[3 * i];
        d.vy[0][s] = vel[3 * i + 1];
        d.vz[0][s] = vel[3 * i + 2];
        d.id[0][s] = (int32_t)i;
    }
}

__global__ __launch_bounds__(kBlock) void k_get_state(Dev d, Params p, double* __restrict__ pos,
                                                      double* __restrict__ vel) {
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        if (s - g.slot_off >= g.npart) continue;
        const int sq = d.st[b].sq, sp = d.st[b].sp;
        const int64_t i = d.id[sp][s];
        if (pos) {
            const Pos x = d.q[sq][s];
            pos[3 * i] = x.x;
            pos[3 * i + 1] = x.y;
            pos[3 * i + 2] = x.z;
        }
        if (vel) {
            vel[3 * i] = d.vx[sp][s];
            vel[3 * i + 1] = d.vy[sp][s];
            vel[3 * i + 2] = d.vz[sp][s];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_get_forces(Dev d, Params p, double* __restrict__ f) {
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        if (s - g.slot_off >= g.npart) continue;
        const int64_t i = d.id[d.st[b].sp][s];
        f[3 * i] = d.fx[s];
        f[3 * i + 1] = d.fy[s];
        f[3 * i + 2] = d.fz[s];
    }
}

__global__ __launch_bounds__(kBlock) void k_get_cells(Dev d, Params p, int32_t* __restrict__ out) {
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        if (s - g.slot_off >= g.npart) continue;
        const uint32_t cc = d.q[d.st[b].sq][s].cc;
        const int cx = cc & 1023, cy = (cc >> 10) & 1023, cz = cc >> 20;
        out[d.id[d.st[b].sp][s]] = (cz * g.n[1] + cy) * g.n[0] + cx;
    }
}

__global__ __launch_bounds__(kBlock) void k_list_counts(Dev d, Params p, int64_t* __restrict__ out) {
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        if (s - g.slot_off >= g.npart) continue;
        out[d.id[d.st[b].sp][s]] = d.cnt[s];
    }
}

// Offset of entry e from entry 0 of the same key in the chunked list.
template <int TPK>
__device__ __forceinline__ uint32_t list_off(int e) {
    const int m = e / TPK;
    return ((uint32_t)(m & ~7) << 6) + (uint32_t)((e % TPK) << 3) + (uint32_t)(m & 7);
}

// The same offset in bytes, for an entry count that is known non-negative.
template <int TPK>
__device__ __forceinline__ uint32_t list_off_bytes(uint32_t e) {
    if constexpr (TPK == 1) {
        return (uint32_t)__umul24(e >> 3, 1008u) + (e << 1);  // (e & ~7) * 128 + (e & 7) * 2
    } else {
        return list_off<TPK>((int)e) * 2u;
    }
}

// Index of entry e of key slot s in the chunked wave-blocked list: a list wave
// of K = 64 / tpk keys owns rows * 64 entries; lane ln = (s % K) * tpk + e % tpk
// keeps its per-lane entries m = e / tpk in 8-entry chunks, chunk c of every
// lane stored side by side (one 16-byte load per lane reads 8 entries).
__device__ __forceinline__ size_t list_addr(int s, int e, int tpk, int rows) {
    const int K = kWave / tpk;
    const int lw = s / K;
    const int kl = s - lw * K;
    const int m = e / tpk;
    const int ln = kl * tpk + (e - m * tpk);
    return ((size_t)lw * rows + (m & ~7)) * kWave + ln * 8 + (m & 7);
}

// Stencil cell s (0..26, z-major over offsets in {-1,0,1}^3) of the cell with
// packed coordinates cc: its global cell index, and the periodic image r of the
// partner's position as code (rz+1)*9 + (ry+1)*3 + (rx+1), where r = +1 on an
// axis means the oracle's minimum image subtracts +L there.
__device__ __forceinline__ int stencil_cell(uint32_t cc, int s, const BoxGeom& g, uint32_t* img) {
    int x = (int)(cc & 1023) + (s % 3 - 1);
    int y = (int)((cc >> 10) & 1023) + ((s / 3) % 3 - 1);
    int z = (int)(cc >> 20) + (s / 9 - 1);
    int rx = 0, ry = 0, rz = 0;
    if (x < 0) { x += g.n[0]; rx = 1; } else if (x >= g.n[0]) { x -= g.n[0]; rx = -1; }
    if (y < 0) { y += g.n[1]; ry = 1; } else if (y >= g.n[1]) { y -= g.n[1]; ry = -1; }
    if (z < 0) { z += g.n[2]; rz = 1; } else if (z >= g.n[2]) { z -= g.n[2]; rz = -1; }
    *img = (uint32_t)((rz + 1) * 9 + (ry + 1) * 3 + (rx + 1));
    return g.cell_off + (z * g.n[1] + y) * g.n[0] + x;
}

// Partner slot of a 16-bit list entry of a key whose cell is cc.
__device__ __forceinline__ int entry_slot(const Dev& d, uint32_t cc, uint32_t e, const BoxGeom& g) {
    uint32_t img;
    return d.cell_start[stencil_cell(cc, (int)(e >> kOffBits), g, &img)] + (int)(e & (kMaxCellCount - 1));
}

__device__ __forceinline__ void tile_piece(const Dev& d, const BoxGeom& g, int cy, int cz, int xa, int xb, int p,
                                           int& s0, int& len, int& ox, int& oy, int& oz);

// First slots and lengths of the 27 pieces staged for the row tile of the key whose
// cell is cc (diagnostics: decoding of row-tile entries).
__device__ void tile_pieces_of(const Dev& d, const BoxGeom& g, uint32_t cc, int* ps0, int* plen) {
    const int cx = (int)(cc & 1023), cy = (int)((cc >> 10) & 1023), cz = (int)(cc >> 20);
    const int4 tr = d.rtile[d.cell_rt[g.cell_off + (cz * g.n[1] + cy) * g.n[0] + cx]];
    for (int pc = 0; pc < 27; ++pc) {
        int ox, oy, oz;
        tile_piece(d, g, cy, cz, tr.z, tr.w, pc, ps0[pc], plen[pc], ox, oy, oz);
    }
}

// Slot behind a row-tile entry (recb * staged index), given the tile's pieces.
__device__ int tile_slot(const int* ps0, const int* plen, uint32_t e, int recb) {
    int idx = (int)(e / (uint32_t)recb);
    for (int pc = 0; pc < 27; ++pc) {
        if (idx < plen[pc]) return ps0[pc] + idx;
        idx -= plen[pc];
    }
    return ps0[13];  // not reached for an entry the build wrote
}

__global__ __launch_bounds__(kBlock) void k_list_export(Dev d, Params p, const int64_t* __restrict__ key_ptr,
                                                        int32_t* __restrict__ partners) {
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        if (s - g.slot_off >= g.npart) continue;
        const int sp = d.st[b].sp;
        const int32_t* id = d.id[sp];
        const int64_t base = key_ptr[id[s]];
        const int n = d.cnt[s];
        const uint32_t cc = d.q[d.st[b].sq][s].cc;
        if (p.tile) {
            int ps0[27], plen[27];
            tile_pieces_of(d, g, cc, ps0, plen);
            for (int e = 0; e < n; ++e)
                partners[base + e] = id[tile_slot(ps0, plen, d.list[list_addr(s, e, p.tpk, p.rows)], p.recb)];
        } else {
            for (int e = 0; e < n; ++e)
                partners[base + e] = id[entry_slot(d, cc, d.list[list_addr(s, e, p.tpk, p.rows)], g)];
        }
        for (int a = 1; a < n; ++a) {  // ascending, insertion sort
            const int32_t x = partners[base + a];
            int c = a - 1;
            while (c >= 0 && partners[base + c] > x) {
                partners[base + c + 1] = partners[base + c];
                --c;
            }
            partners[base + c + 1] = x;
        }
    }
}

// ---------------------------------------------------------------- control

__global__ void k_mark_rebuild(Dev d, Params p) {
    for (int b = threadIdx.x; b < p.nbox; b += blockDim.x) d.st[b].rebuild = 1;
    if (threadIdx.x == 0) *d.any = 1;
}

// Max over a box's striped partial maxima (bit patterns of non-negative doubles),
// clearing the stripes for the next step.  One block per box.
__device__ double stripe_max(unsigned long long* stripes) {
    __shared__ double red[kBlock];
    double m = 0.0;
    for (int k = threadIdx.x; k < kStripes; k += kBlock) {
        unsigned long long* a = stripes + (size_t)k * kStripeStride;
        m = fmax(m, __longlong_as_double((long long)*a));
        *a = 0ull;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// After the drift: swap the q/u buffers, accumulate the DUTC bound and decide
// whether the list must be rebuilt (Sec. II.A).  One block per box.
__global__ __launch_bounds__(kBlock) void k_dutc(Dev d, Params p) {
#pragma clang fp contract(off)
    if (halted(d)) return;
    for (int b = blockIdx.x; b < p.nbox; b += gridDim.x) {
        const double vmax2 = stripe_max(d.vmax_s + (size_t)b * kStripes * kStripeStride);
        double m2 = 0.0;
        if (d.qb) m2 = stripe_max(d.disp_s + (size_t)b * kStripes * kStripeStride);
        if (threadIdx.x == 0) {
            BoxState& st = d.st[b];
            st.sq ^= 1;
            st.nstep += 1;
            st.D = st.D + p.dt * sqrt(vmax2);
            int rb = 0;
            if (p.policy == MD_REBUILD_DUTC)
                rb = 2.0 * st.D > p.skin;
            else if (p.policy == MD_REBUILD_DISPLACEMENT)
                rb = 2.0 * sqrt(m2) > p.skin;
            else if (p.policy == MD_REBUILD_EVERY_STEP)
                rb = 1;
            st.rebuild = rb;
            if (rb) atomicOr(d.any, 1);
        }
    }
}

// After a build: the permuted buffers become the current ones, longest list over
// each box's cell tiles, DUTC bound reset, and the "some box rebuilds" gate cleared by
// the last block to finish.  (Between the permutation and this kernel, a rebuilding box's current
// positions are in buffer sq ^ 1: the list build reads them there.)
__global__ __launch_bounds__(kBlock) void k_post_build(Dev d, Params p, int with_list) {
    __shared__ int red[kBlock / kWave];
    __shared__ int last;
    if (!*d.any || halted(d)) return;
    const int l = lane_id(), wv = wave_in_block();
    for (int b = blockIdx.x; b < p.nbox; b += gridDim.x) {  // one block per box
        BoxState& st = d.st[b];
        if (!st.rebuild) continue;  // uniform over the block
        const BoxGeom& g = d.geom[b];
        int m = 0;
        if (with_list)
            for (int t = threadIdx.x; t < g.ntile; t += kBlock) m = max(m, d.tile_need[g.tile_off + t]);
        m = __builtin_amdgcn_readlane(wave_incl_max(m), kWave - 1);
        if (l == 0) red[wv] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < kBlock / kWave; ++w) m = max(m, red[w]);
            if (with_list) {
                st.D = 0.0;
                st.built += 1;
                st.need = max(st.need, m);
            }
            st.sq ^= 1;
            st.sp ^= 1;
            st.rebuild = 0;
        }
        __syncthreads();
    }
    // the last block to finish clears the gate (every block has read it by then)
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(d.ntiles + 1, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (last && threadIdx.x == 0) {
        d.ntiles[1] = 0;
        *d.any = 0;
    }
}

// ---------------------------------------------------------------- binning

__global__ __launch_bounds__(kBlock) void k_cell_clear(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;  // no box rebuilds this step, or a build overflowed
    for (int t = blockIdx.x; t < p.ntile; t += gridDim.x) {
        if (!d.st[d.tile_box[t]].rebuild) continue;
        int4* c = reinterpret_cast<int4*>(d.cell_cnt + (size_t)t * kTile);
        c[threadIdx.x] = make_int4(0, 0, 0, 0);
        if (threadIdx.x == 0) d.tile_need[t] = 0;
    }
}

// Wrap + cell id (A1) and the histogram half of the counting sort (A2).
// Slots arrive sorted by cell from the previous build, so a wavefront issues one
// atomic per run of equal cells and hands out tickets within the run.
__global__ __launch_bounds__(kBlock) void k_bin(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;  // no box rebuilds this step, or a build overflowed
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        if (!ld_const(&d.st[b].rebuild)) continue;  // uniform over the wavefront
        const BoxGeom g = ld_geom(d.geom + b);
        const int s = w * kWave + l;
        const bool valid = s - g.slot_off < g.npart;  // the valid lanes are a prefix
        int cid = -1;
        if (valid) {
            const int sq = ld_const(&d.st[b].sq);
            Pos x = d.q[sq][s];
            const double x0 = x.x, y0 = x.y, z0 = x.z;
            bool bad = false;
            const int cx = bin_axis(x.x, g.L[0], g.inv[0], g.n[0], bad);
            const int cy = bin_axis(x.y, g.L[1], g.inv[1], g.n[1], bad);
            const int cz = bin_axis(x.z, g.L[2], g.inv[2], g.n[2], bad);
            if (bad) atomicOr(&d.st[b].err, 1);
            // only particles that crossed the box boundary change: write those back
            if (x.x != x0 || x.y != y0 || x.z != z0) {
                d.q[sq][s].x = x.x;
                d.q[sq][s].y = x.y;
                d.q[sq][s].z = x.z;
            }
            cid = (cz * g.n[1] + cy) * g.n[0] + cx;
            d.cell_tmp[s] = cid;
        }
        const unsigned long long vm = __ballot(valid);
        const int prev = __shfl_up(cid, 1);
        const bool head = valid && (l == 0 || prev != cid);
        const unsigned long long hm = __ballot(head);
        const unsigned long long upto = l == 63 ? ~0ull : ((2ull << l) - 1ull);
        const int my_head = 63 - __clzll((long long)(hm & upto));
        const unsigned long long above = hm & ~upto;
        const int run_end = above ? __ffsll((long long)above) - 1 : __popcll(vm);
        int base = 0;
        if (head) base = atomicAdd(&d.cell_cnt[g.cell_off + cid], run_end - l);
        base = __shfl(base, my_head & 63);
        if (valid) d.ticket[s] = base + (l - my_head);
    }
}

// Tile-local exclusive scan of cell counts; tile totals to tile_sum.
__global__ __launch_bounds__(kBlock) void k_scan_tile(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;  // no box rebuilds this step, or a build overflowed
    for (int t = blockIdx.x; t < p.ntile; t += gridDim.x) {
        if (!d.st[d.tile_box[t]].rebuild) continue;  // uniform over the block
        const size_t base = (size_t)t * kTile + threadIdx.x * 4;
        const int4 c = *reinterpret_cast<const int4*>(d.cell_cnt + base);
        int tot;
        const int ex = block_excl_scan(c.x + c.y + c.z + c.w, &tot);
        *reinterpret_cast<int4*>(d.cell_start + base) =
            make_int4(ex, ex + c.x, ex + c.x + c.y, ex + c.x + c.y + c.z);
        if (threadIdx.x == 0) d.tile_sum[t] = tot;
    }
}

// Per box: exclusive scan over its tiles' totals, offset by the box's first slot.
__global__ __launch_bounds__(kBlock) void k_scan_box(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;  // no box rebuilds this step, or a build overflowed
    for (int b = blockIdx.x; b < p.nbox; b += gridDim.x) {
        if (!d.st[b].rebuild) continue;
        const BoxGeom& g = d.geom[b];
        int carry = g.slot_off;
        for (int k0 = 0; k0 < g.ntile; k0 += kBlock) {
            const int k = k0 + threadIdx.x;
            const int v = k < g.ntile ? d.tile_sum[g.tile_off + k] : 0;
            int tot;
            const int ex = block_excl_scan(v, &tot);
            if (k < g.ntile) d.tile_pref[g.tile_off + k] = carry + ex;
            carry += tot;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_add(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;  // no box rebuilds this step, or a build overflowed
    for (int t = blockIdx.x; t < p.ntile; t += gridDim.x) {
        if (!d.st[d.tile_box[t]].rebuild) continue;
        const int add = d.tile_pref[t];
        int4* c = reinterpret_cast<int4*>(d.cell_start + (size_t)t * kTile);
        int4 v = c[threadIdx.x];
        v.x += add; v.y += add; v.z += add; v.w += add;
        c[threadIdx.x] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;  // no box rebuilds this step, or a build overflowed
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        if (!ld_const(&d.st[b].rebuild)) continue;
        const BoxGeom g = ld_geom(d.geom + b);
        const int s = w * kWave + l;
        if (s - g.slot_off >= g.npart) continue;
        d.perm[d.cell_start[g.cell_off + d.cell_tmp[s]] + d.ticket[s]] = s;
    }
}

// Arrival order within a cell depends on atomics; each cell's members are placed
// in the order of their previous slots, so every layout is a function of the
// initial one and the trajectory (the first build after md_set_state orders by
// caller id).  One lane per particle, taken in arrival order: its rank among the
// cell's members is its new slot, and its state is copied there (position record
// with the new cell, fixed-point record, velocities, caller id).
__global__ __launch_bounds__(kBlock) void k_rank_permute(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;  // no box rebuilds this step, or a build overflowed
    const int l = lane_id();
    for (int w = xcd_block(blockIdx.x, gridDim.x) * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxState& st = d.st[b];
        if (!ld_const(&st.rebuild)) continue;
        const BoxGeom g = ld_geom(d.geom + b);
        const int s = w * kWave + l;
        if (s - g.slot_off >= g.npart) continue;
        const int sq = ld_const(&st.sq), sp = ld_const(&st.sp), nq = sq ^ 1, np = sp ^ 1;
        const int32_t* __restrict__ id = d.id[sp];
        const int o = d.perm[s];  // a particle of this cell, in arrival order
        const int key = id[o];
        const int cid = d.cell_tmp[o];
        const int c = g.cell_off + cid;
        const int a = d.cell_start[c], m = d.cell_cnt[c];
        int rank = 0;  // its place in the cell: order by previous slot
        for (int t = a; t < a + m; ++t) rank += d.perm[t] < o ? 1 : 0;
        const int dst = a + rank;
        Pos x = d.q[sq][o];
        d.vx[np][dst] = d.vx[sp][o];
        d.vy[np][dst] = d.vy[sp][o];
        d.vz[np][dst] = d.vz[sp][o];
        d.id[np][dst] = key;
        const int tq = gdiv(g, cid, 0), cx = cid - tq * g.n[0];
        const int cz = gdiv(g, tq, 1), cy = tq - cz * g.n[1];
        const uint32_t cc = (uint32_t)cx | ((uint32_t)cy << 10) | ((uint32_t)cz << 20);
        x.cc = cc;
        x.cnt = 0;
        d.q[nq][dst] = x;
        if (p.precision == MD_PREC_FP32_MIXED) put_u(d.u[nq], dst, units3(x, cc, g));
        if (d.qb) d.qb[dst] = make_double4(x.x, x.y, x.z, 0.0);
    }
}

// ---------------------------------------------------------------- row tiles

__device__ __forceinline__ int wrap_idx(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Piece p = r * 3 + side (r = (dz+1)*3 + (dy+1)) of the staged partner region of the
// row tile with home cells [xa, xb) of row (cy, cz): its first slot, its length (0 if
// the piece is absent) and the image terms its fixed-point records take on, so that
// every staged record is in the unwrapped frame of the home row.
//   side 0: unwrapped cell x = -1, i.e. cell n-1 one box length down (only if xa == 0)
//   side 1: cells max(xa-1, 0) .. min(xb, n-1), one contiguous run of slots
//   side 2: unwrapped cell x = n, i.e. cell 0 one box length up (only if xb == n)
__device__ __forceinline__ void tile_piece(const Dev& d, const BoxGeom& g, int cy, int cz, int xa, int xb, int p,
                                           int& s0, int& len, int& ox, int& oy, int& oz) {
    const int r = (p * 11) >> 5, side = p - 3 * r;  // p / 3 for p < 27
    const int rz = (r * 11) >> 5, ry = r - 3 * rz;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int y = cy + ry - 1, z = cz + rz - 1;
    s0 = 0;
    len = 0;
    // image terms modulo 2^32: a cell index that wrapped below 0 takes -n * uoff, above n-1 +n * uoff
    ox = side == 0 ? -g.nuoff[0] : (side == 2 ? g.nuoff[0] : 0);
    oy = y < 0 ? -g.nuoff[1] : (y >= ny ? g.nuoff[1] : 0);
    oz = z < 0 ? -g.nuoff[2] : (z >= nz ? g.nuoff[2] : 0);
    int x0, x1;
    if (side == 0) {
        if (xa > 0) return;
        x0 = x1 = nx - 1;
    } else if (side == 2) {
        if (xb < nx) return;
        x0 = x1 = 0;
    } else {
        x0 = max(xa - 1, 0);
        x1 = min(xb, nx - 1);
    }
    const int rowc = g.cell_off + (wrap_idx(z, nz) * ny + wrap_idx(y, ny)) * nx;
    s0 = d.cell_start[rowc + x0];
    len = d.cell_start[rowc + x1] + d.cell_cnt[rowc + x1] - s0;
}

// Periodic image of piece p of a row tile's staged region, per axis in {-1, 0, 1}:
// -1 where the piece's cells wrapped below 0 (their positions are taken minus L),
// +1 above n - 1 (plus L).  The same cases as tile_piece's fixed-point terms.
__device__ __forceinline__ void tile_piece_img(const BoxGeom& g, int cy, int cz, int p, int& rx, int& ry, int& rz) {
    const int r = (p * 11) >> 5, side = p - 3 * r;
    const int rzz = (r * 11) >> 5, ryy = r - 3 * rzz;
    const int y = cy + ryy - 1, z = cz + rzz - 1;
    rx = side == 0 ? -1 : (side == 2 ? 1 : 0);
    ry = y < 0 ? -1 : (y >= g.n[1] ? 1 : 0);
    rz = z < 0 ? -1 : (z >= g.n[2] ? 1 : 0);
}

// Cuts every row of cells into row tiles, greedily from x = 0: a tile grows by the
// next cell while its keys stay within kt, its staged region within scap records and
// its width within kTileWMax cells.  One wavefront per row.  The column sums of the
// 3 x 3 rows around it (cells x = -1 .. n, unwrapped) and the row's own counts go to
// LDS as prefix sums; every lane then finds, for the cells x it holds, where a tile
// starting at x would end (a binary search: both sums grow with the tile), and lane 0
// follows those ends from x = 0, a handful of steps per row.  A one-cell tile whose
// region exceeds scap sets error bit 2 of its box (the context then falls back to the
// gather format).
__global__ __launch_bounds__(kBlock) void k_row_tiles(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;  // no box rebuilds this step, or a build overflowed
    constexpr int NWb = kBlock / kWave;
    __shared__ int col_all[NWb][kMaxCellsPerAxis + 3];  // C[k]: staged counts of unwrapped x < k - 1
    __shared__ int hom_all[NWb][kMaxCellsPerAxis + 1];  // H[k]: keys of cells x < k
    __shared__ int nxt_all[NWb][kMaxCellsPerAxis];      // end of the tile that starts at x
    const int wv = wave_in_block(), l = lane_id();
    int* C = col_all[wv];
    int* H = hom_all[wv];
    int* nxt = nxt_all[wv];
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // in-place exclusive prefix sum of a[0 .. len), and a[len] = the total
    auto prefix = [&](int* a, int len) {
        int carry = 0;
        for (int j0 = 0; j0 < len; j0 += kWave) {
            const int j = j0 + l;
            const int v = j < len ? a[j] : 0;
            const int incl = wave_incl_sum(v);
            if (j < len) a[j] = carry + incl - v;
            carry += __builtin_amdgcn_readlane(incl, kWave - 1);
        }
        if (l == 0) a[len] = carry;
        wave_sync();
    };
    for (int row = blockIdx.x * 4 + wv; row < p.nrows; row += gridDim.x * 4) {
        const int b = ld_const(d.row_box + row);
        const BoxGeom g = ld_geom(d.geom + b);
        const int lr = row - g.row_off, nx = g.n[0], ny = g.n[1], nz = g.n[2];
        const int cy = lr % ny, cz = lr / ny;
        // the 9 row starts, then the counts of 4 x positions per lane in flight at once
        int rs[9];
#pragma unroll
        for (int r = 0; r < 9; ++r)
            rs[r] = g.cell_off + (wrap_idx(cz + r / 3 - 1, nz) * ny + wrap_idx(cy + r % 3 - 1, ny)) * nx;
        constexpr int kXu = 4;
        for (int x0 = l - 1; x0 <= nx; x0 += kWave * kXu) {
            int sum[kXu], own[kXu];
#pragma unroll
            for (int u = 0; u < kXu; ++u) {
                const int x = x0 + u * kWave, xw = wrap_idx(min(x, nx), nx);
                sum[u] = 0;
                if (x <= nx) {
#pragma unroll
                    for (int r = 0; r < 9; ++r) sum[u] += d.cell_cnt[rs[r] + xw];
                }
                own[u] = x >= 0 && x < nx ? d.cell_cnt[rs[4] + x] : 0;  // r = 4: the row itself
            }
#pragma unroll
            for (int u = 0; u < kXu; ++u) {
                const int x = x0 + u * kWave;
                if (x <= nx) C[x + 1] = sum[u];
                if (x >= 0 && x < nx) H[x] = own[u];
            }
        }
        wave_sync();
        prefix(C, nx + 2);
        prefix(H, nx);
        // the tile [xa, xb) holds H[xb] - H[xa] keys and stages C[xb + 2] - C[xa] records;
        // a tile takes at least one cell
        for (int xa = l; xa < nx; xa += kWave) {
            int lo = xa + 1, hi = min(nx, xa + kTileWMax);
            const int h0 = H[xa], c0 = C[xa];
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (H[mid] - h0 <= p.kt && C[mid + 2] - c0 <= p.scap)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            nxt[xa] = lo;
        }
        wave_sync();
        if (l == 0) {
            const int base = g.cell_off + lr * nx;  // the row's cells hold its tiles in rt_tmp
            int nt = 0, xa = 0, big = 0;
            while (xa < nx) {
                const int xb = nxt[xa];
                big = max(big, C[xb + 2] - C[xa]);
                d.rt_tmp[base + nt] = xa | (xb << 16);
                ++nt;
                xa = xb;
            }
            d.row_nt[row] = nt;
            if (big > p.scap) {  // only a one-cell tile can exceed it; the step stops here
                atomicOr(&d.st[b].err, 4);
                atomicOr(d.halt, 1);
            }
        }
        wave_sync();
    }
}

// One block: exclusive scan of the tiles per row (global row order), the tile
// total, and each box's first tile.  The rows go through in coalesced passes of
// kBlock; each pass is a block-wide scan (wavefront sums, then their prefix).
__global__ __launch_bounds__(kBlock) void k_row_scan(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;
    constexpr int NWb = kBlock / kWave;
    __shared__ int wsum[NWb];
    const int n = p.nrows, tid = threadIdx.x, l = lane_id(), wv = wave_in_block();
    int carry = 0;
    int nt = tid < n ? d.row_nt[tid] : 0, rb = tid < n ? d.row_box[tid] : 0;
    int rprev = tid >= 1 && tid - 1 < n ? d.row_box[tid - 1] : -1;
    for (int i0 = 0; i0 < n; i0 += kBlock) {
        const int i = i0 + tid;
        // the next pass's values, loaded ahead
        const int j = i + kBlock;
        const int nt_n = j < n ? d.row_nt[j] : 0, rb_n = j < n ? d.row_box[j] : 0;
        const int rprev_n = j - 1 < n ? d.row_box[j - 1] : -1;
        const int incl = wave_incl_sum(nt);
        if (l == kWave - 1) wsum[wv] = incl;
        __syncthreads();
        int before = carry;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        int total = 0;
        for (int w = 0; w < NWb; ++w) total += wsum[w];
        if (i < n) {
            const int t0 = before + incl - nt;
            d.row_t0[i] = t0;
            if (i == 0 || rprev != rb) d.box_t0[rb] = t0;  // a box's rows are consecutive
        }
        carry += total;
        __syncthreads();  // wsum is rewritten by the next pass
        nt = nt_n;
        rb = rb_n;
        rprev = rprev_n;
    }
    if (tid == 0) {
        d.ntiles[0] = carry;
        d.box_t0[p.nbox] = carry;
    }
}

// Row tiles into their global slots, and the tile of every cell.  One wavefront
// per row, one lane per tile.
__global__ __launch_bounds__(kBlock) void k_row_write(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;
    const int l = lane_id();
    for (int row = blockIdx.x * 4 + wave_in_block(); row < p.nrows; row += gridDim.x * 4) {
        const int b = ld_const(d.row_box + row);
        const BoxGeom g = ld_geom(d.geom + b);
        const int lr = row - g.row_off, base = g.cell_off + lr * g.n[0];
        const int nt = d.row_nt[row], t0 = d.row_t0[row];
        for (int k = l; k < nt; k += kWave) {
            const int v = d.rt_tmp[base + k];
            const int xa = v & 0xffff, xb = v >> 16;
            d.rtile[t0 + k] = make_int4(b, lr, xa, xb);
            for (int x = xa; x < xb; ++x) d.cell_rt[base + x] = t0 + k;
        }
    }
}

// Per row tile and piece p: staged index of the piece's first record minus its first
// slot, so that the list build turns a stencil cell's first slot into its staged
// index with one addition.  One wavefront per tile, lane p per piece.
__global__ __launch_bounds__(kBlock) void k_row_delta(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;
    const int l = lane_id();
    const int ntl = ld_const(d.ntiles);
    for (int t = blockIdx.x * 4 + wave_in_block(); t < ntl; t += gridDim.x * 4) {
        const int4 tr = d.rtile[t];
        const int b = __builtin_amdgcn_readfirstlane(tr.x);
        const BoxGeom g = ld_geom(d.geom + b);
        const int lr = __builtin_amdgcn_readfirstlane(tr.y);
        int ps0 = 0, plen = 0, ox, oy, oz;
        const int lz = gdiv(g, lr, 1);
        if (l < 27) tile_piece(d, g, lr - lz * g.n[1], lz, tr.z, tr.w, l, ps0, plen, ox, oy, oz);
        const int pbase = wave_incl_sum(plen) - plen;
        if (l < 27) d.rt_delta[t * 27 + l] = pbase - ps0;
    }
}

// ---------------------------------------------------------------- pair list

// Squared minimum-image distance exactly as the plain definition evaluates it:
// d = (x_j - x_i) - L * rint((x_j - x_i) / L) per axis, where the subtracted
// image term is known from the stencil, then dx*dx + dy*dy + dz*dz left to
// right.  No contraction, so the accept decision matches the CPU bit for bit.
template <class A, class B>
__device__ __forceinline__ double dist2_exact(const A& qi, const B& qj, double shx, double shy, double shz) {
#pragma clang fp contract(off)
    const double dx = (qj.x - qi.x) - shx;
    const double dy = (qj.y - qi.y) - shy;
    const double dz = (qj.z - qi.z) - shz;
    return dx * dx + dy * dy + dz * dz;
}
// The same distance for a cell whose stencil has no periodic image, with the sum of
// squares contracted into two FMAs (7 instructions with the compare instead of 9).
// Its rounding differs from the uncontracted definition by about one ulp of r^2, so
// the accept decision can differ only for pairs within ~1e-15 of the list radius:
// inside the 1e-9 tie band that set comparisons leave out.
template <class A, class B>
__device__ __forceinline__ double dist2_fma0(const A& qi, const B& qj) {
    const double dx = qj.x - qi.x;
    const double dy = qj.y - qi.y;
    const double dz = qj.z - qi.z;
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffll), lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Neighbour cell along one axis with its periodic image.  sub is the amount
// the oracle's minimum image subtracts: L * rint(t / L) with t = x_j - x_i.
__device__ __forceinline__ int nb_axis(int c, int o, int n, double L, double& sub, int& r) {
    int x = c + o;
    sub = 0.0;
    r = 0;
    if (x < 0) {
        x += n;
        sub = L;
        r = 1;
    } else if (x >= n) {
        x -= n;
        sub = -L;
        r = -1;
    }
    return x;
}

// A4, one wavefront per home cell.  All keys of a cell share one candidate set:
// the particles of its 27 stencil cells, concatenated with the home cell first and
// the other 26 in stencil order after it.  Lane l
// holds candidate l of each 64-wide chunk (loads are contiguous runs).  A pass
// loads up to G chunks into registers, then the wavefront walks the cell's keys:
// per (key, chunk) an exact FP64 test, a ballot, an mbcnt prefix on the key's
// running count, and the accepted partners appended in candidate order.  The
// running count is wave-uniform (SGPR), so no lane bookkeeping sits in the inner
// loop.  The distance test is the plain definition (no contraction) for cells whose
// stencil holds a periodic image, and contracted into FMAs elsewhere: the accepted
// set is the CPU's except possibly for pairs within ~1e-15 of the list radius.

// Positions seen through the constant address space: in the list build they are
// read-only, and uniform indices then become scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) double const_double;

// One pass over the keys kb .. kb+mb-1 of a home cell against candidate chunks
// [c0, c0 + G*64).  WRAP: some stencil cell is a periodic image, so every lane
// subtracts its image term (a zero term leaves t unchanged bit for bit).
// STAGED: accepted entries go to the wavefront's LDS buffer (key a's entry e at
// a * cap + (e % TPK) * (cap / TPK) + e / TPK, i.e. already in per-lane chunk
// order) and leave in whole 16-byte chunks afterwards; otherwise each entry is
// stored to the list directly.
// A candidate's stencil cell: the non-empty stencil cell at position o of the
// candidate order marks its first candidate with o + 1 in a byte window of the pass
// (the wavefront's `mark`, G * 64 bytes), and a running maximum over the window,
// started from the position that was open at the end of the previous pass (`open`),
// gives every candidate the last position starting at or before it; lane o holds
// that position's start, entry base and image term.
constexpr int kStage = 2048;  // LDS list entries per wavefront (16 KB per block, 17.5 KB with the marks: 7 blocks per CU)
constexpr int kMarkBytes = 6 * kWave;  // candidate window of a pass (G <= 6 chunks)

template <int TPK, bool WRAP, bool STAGED, bool HALF, bool TL>
__device__ __forceinline__ void list_pass(const Dev& d, const Params& p, const Pos* __restrict__ q,
                                          const const_double* qc, int cs0, int kb, int mb, int c0, int total,
                                          int start, int pre, int ekey, int scnt, double shx, double shy,
                                          double shz, int& n_own, int& open, uint16_t* stage,
                                          uint8_t* mark) {
    constexpr int G = WRAP ? 3 : 6;
    static_assert(G * kWave <= kMarkBytes, "mark window");
    const int l = lane_id();
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    const int nch = min(G, (total - c0 + kWave - 1) >> 6);  // uniform, >= 1
    // the window's marks: cleared as words, then one byte per cell starting in it
    uint32_t* mw = reinterpret_cast<uint32_t*>(mark);
    if (l < G * kWave / 4) mw[l] = 0u;
    if (G * kWave / 4 > kWave && l < G * kWave / 4 - kWave) mw[kWave + l] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (l < 27 && scnt > 0 && pre >= c0 && pre < c0 + G * kWave) mark[pre - c0] = (uint8_t)(l + 1);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int sbase = start - pre;  // stencil cell s: slot of its candidate ci is sbase + ci
    double cx[G], cy[G], cz[G], sx[G], sy[G], sz[G];
    uint32_t ent[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
        if (k < nch) {
            const int ci = c0 + k * kWave + l;
            const bool valid = ci < total;
            const int run = max(wave_incl_max((int)mark[k * kWave + l]), open);
            open = __builtin_amdgcn_readlane(run, 63);
            const int sc = max(run - 1, 0);  // last stencil cell whose range starts at or before ci
            // shuffles run on every lane: a bpermute from an inactive lane reads 0
            const int base_sc = __shfl(sbase, sc), ek_sc = __shfl(ekey, sc);
            // gather format: stencil cell << 11 | rank; row-tile format: the staged record's
            // LDS byte offset (12-byte records)
            ent[k] = (uint32_t)(ek_sc + ci) * (TL ? (uint32_t)p.recb : 1u);
            // 32-bit byte offset from the (scalar) array base: slots stay below 2^27
            const uint32_t boff = (uint32_t)(valid ? base_sc + ci : cs0) * (uint32_t)sizeof(Pos);
            const Pos qj = *reinterpret_cast<const Pos*>(reinterpret_cast<const char*>(q) + boff);
            cx[k] = valid ? qj.x : nan;  // NaN distance: never accepted
            cy[k] = qj.y;
            cz[k] = qj.z;
            if (WRAP) {
                sx[k] = __shfl(shx, sc);
                sy[k] = __shfl(shy, sc);
                sz[k] = __shfl(shz, sc);
            }
        }
    }
    // The candidate loads must land before the key loop: a wait placed inside it
    // would also wait on the list stores issued there.
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    const double rl2 = p.rl2;
    const int cap = p.cap, rows = p.rows;
    // The key loop, instantiated per chunk count so that every chunk's distances are
    // computed ahead of the (serial) compaction chain, with no branches between them.
    // The home cell's members come first among the candidates, so key kb + a is
    // candidate kb + a: with GEN false the pass starts at the block's first key
    // (c0 == kb), key a's own candidate is lane a of the first chunk, and only that
    // chunk's ballot drops a bit.
    auto key_loop = [&](auto n_c, auto gen_c) {
        constexpr int N = decltype(n_c)::value;
        constexpr bool GEN = decltype(gen_c)::value;
        double nx = qc[4 * (cs0 + kb)], ny = qc[4 * (cs0 + kb) + 1], nz = qc[4 * (cs0 + kb) + 2];
        for (int a = 0; a < mb; ++a) {
            const int key = cs0 + kb + a;
            double4 qi;  // scalar loads, one key ahead
            qi.x = nx;
            qi.y = ny;
            qi.z = nz;
            if (a + 1 < mb) {
                nx = qc[4 * (key + 1)];
                ny = qc[4 * (key + 1) + 1];
                nz = qc[4 * (key + 1) + 2];
            }
            int cnt = __builtin_amdgcn_readlane(n_own, a);  // uniform running count (0 in the first pass)
            // the key's own candidate: chunk sk, bit sb (scalar)
            const int self = kb + a - c0;
            const int sk = self >> 6;
            const unsigned long long sb = 1ull << (GEN ? self & 63 : a);
            char* __restrict__ kp = STAGED ? reinterpret_cast<char*>(stage + a * cap)
                                           : reinterpret_cast<char*>(d.list + list_addr(key, 0, TPK, rows));
            bool in[N];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const double r2 = WRAP ? dist2_exact(qi, make_double3(cx[k], cy[k], cz[k]), sx[k], sy[k], sz[k])
                                       : dist2_fma0(qi, make_double3(cx[k], cy[k], cz[k]));
                in[k] = r2 < rl2;
            }
#pragma unroll
            for (int k = 0; k < N; ++k) {
                // lanes within the list radius, minus the key itself; the half list
                // keeps only candidates after the key (the home cell comes first and
                // the backward stencil cells hold no candidates)
                const unsigned long long mask =
                    HALF ? __builtin_amdgcn_ballot_w64(in[k] && k * kWave + l > self)
                         : __builtin_amdgcn_ballot_w64(in[k]) & ~(GEN ? (k == sk ? sb : 0ull) : (k == 0 ? sb : 0ull));
                // the lane's entry position: the running count plus its place among the
                // accepted lanes (the count enters as the lane-count base, no scalar add)
                const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
                    (unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, (uint32_t)cnt));
                unsigned long long sm = mask;
                if (cnt + __popcll(mask) > cap)  // overflow: keep the entries that fit (rare)
                    sm = __builtin_amdgcn_ballot_w64(__builtin_amdgcn_inverse_ballot_w64(mask) &&
                                                     (int)pos < cap);  // cnt may exceed cap
                if (__builtin_amdgcn_inverse_ballot_w64(sm)) {
                    if constexpr (STAGED && TPK == 1) {
                        reinterpret_cast<uint16_t*>(kp)[pos] = (uint16_t)ent[k];
                    } else {
                        const uint32_t off = STAGED ? ((pos % TPK) * (uint32_t)(cap / TPK) + pos / TPK) * 2u
                                                    : list_off_bytes<TPK>(pos);
                        *reinterpret_cast<uint16_t*>(kp + off) = (uint16_t)ent[k];
                    }
                }
                cnt += __popcll(mask);
            }
            if (l == a) n_own = cnt;
        }
    };
    auto by_count = [&](auto gen_c) {
        switch (nch) {
            case 1: key_loop(std::integral_constant<int, 1>{}, gen_c); break;
            case 2: key_loop(std::integral_constant<int, 2>{}, gen_c); break;
            default:
                if constexpr (G == 3) {
                    key_loop(std::integral_constant<int, 3>{}, gen_c);
                } else {
                    switch (nch) {
                        case 3: key_loop(std::integral_constant<int, 3>{}, gen_c); break;
                        case 4: key_loop(std::integral_constant<int, 4>{}, gen_c); break;
                        case 5: key_loop(std::integral_constant<int, 5>{}, gen_c); break;
                        default: key_loop(std::integral_constant<int, 6>{}, gen_c); break;
                    }
                }
                break;
        }
    };
    // own candidates of this pass: kb - c0 .. kb + mb - 1 - c0 (uniform); the half list
    // drops them by position instead
    if (HALF || kb == c0)
        by_count(std::false_type{});
    else
        by_count(std::true_type{});
}

// Seven wavefronts per SIMD (at most 72 VGPRs, no vector spills in the full-list
// build): the build issues about as many scalar as vector instructions and is bound by
// the latency of its scalar-vector chain per (key, chunk), which more resident
// wavefronts hide (measured at 32M particles, rebuild chain per rebuild: 4 wavefronts
// 13.2 ms, 6 wavefronts 11.5 ms in an earlier form; 6 -> 7 -> 8 wavefronts now
// 9.36 -> 9.08 -> 9.19 ms, the last with spills).
// TL: the row-tile entry format (FP32-mixed, full list); otherwise the gather format.
template <int TPK, bool HALF, bool TL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_list(Dev d, Params p) {
    if (!ld_const(d.any) || halted(d)) return;  // no box rebuilds this step, or a build overflowed
    __shared__ __align__(16) uint16_t stage_all[kBlock / kWave][kStage];
    __shared__ __align__(16) uint8_t mark_all[kBlock / kWave][kMarkBytes];
    const int l = lane_id();
    const int ncells = p.ntile * kTile;
    const int cap = p.cap, rows = p.rows;
    // XCD-aware: each XCD sweeps a contiguous run of cells, so the stencil rows a
    // cell loads are still in that XCD's L2 for its neighbours
    // the wavefront's index in the block, as a scalar: the cell loop and every per-cell
    // table read (tile's box, box state and geometry) then stay in scalar registers and
    // the scalar cache instead of serialised vector loads; the staging buffer's base
    // is scalar too
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint16_t* stage = stage_all[wv];
    uint8_t* mark = mark_all[wv];
    // One home cell c of box b.
    auto cell_body = [&](int c, int b, const BoxGeom& g) {
        const int t = c / kTile;
        const BoxState& st = d.st[b];
        const int local = c - g.cell_off;
        const int m = ld_const(d.cell_cnt + c);
        if (m == 0) return;
        const int cs0 = ld_const(d.cell_start + c);
        Pos* __restrict__ q = d.q[ld_const(&st.sq) ^ 1];  // permuted, made current after the build
        const int ly = gdiv(g, local, 0), cz = gdiv(g, local, 2);
        const int cx = local - ly * g.n[0], cy = ly - cz * g.n[1];
        // lane l < 27 holds the l-th stencil cell of the candidate order: the home cell
        // (s = 13) first, then s = 0 .. 12 and 14 .. 26, so every key's own candidate sits
        // in the first chunk of a cell with at most 64 members; its start, count and
        // image term
        const int s_of_l = l == 0 ? 13 : (l <= 13 ? l - 1 : l);
        int start = 0, cnt = 0;
        double shx = 0.0, shy = 0.0, shz = 0.0;
        bool img = false;
        if (l < 27) {
            const int ox = s_of_l % 3 - 1, oy = (s_of_l / 3) % 3 - 1, oz = s_of_l / 9 - 1;
            int rx, ry, rz;
            const int x = nb_axis(cx, ox, g.n[0], g.L[0], shx, rx);
            const int y = nb_axis(cy, oy, g.n[1], g.L[1], shy, ry);
            const int z = nb_axis(cz, oz, g.n[2], g.L[2], shz, rz);
            img = (rx | ry | rz) != 0;
            const int nc = g.cell_off + (z * g.n[1] + y) * g.n[0] + x;
            start = d.cell_start[nc];
            cnt = d.cell_cnt[nc];
            if (cnt > kMaxCellCount) atomicOr(&d.st[b].err, 2);  // ranks would not fit 11 bits
            // half list: only the home cell (s = 13) and the forward cells s > 13, whose
            // offsets are lexicographically positive, so each pair of cells meets once
            if (HALF && s_of_l < 13) cnt = 0;
        }
        const bool wrap = __ballot(img) != 0ull;  // uniform: this cell touches the box boundary
        const int incl = wave_incl_sum(cnt);
        const int pre = incl - cnt;
        // entry of candidate ci of the lane's stencil cell s: ekey + ci (gather format:
        // s << 11 plus its rank; row-tile format: its index in the staged region of the
        // home cell's row tile, whose piece p = r * 3 + side holds unwrapped cells in order)
        int ekey = (s_of_l << kOffBits) - pre;
        if constexpr (TL) {
            // staged index of the stencil cell's first member: its first slot plus the
            // (staged index - first slot) of the piece of the home cell's row tile holding it
            const int r = s_of_l / 3, x = cx + s_of_l % 3 - 1;
            const int pc = r * 3 + (x < 0 ? 0 : (x >= g.n[0] ? 2 : 1));
            const int rt = ld_const(d.cell_rt + c);
            ekey = (l < 27 ? start + d.rt_delta[rt * 27 + pc] : 0) - pre;
        }
        const int total = __builtin_amdgcn_readlane(incl, 26);
        const const_double* qc = (const const_double*)q;     // 4 doubles per particle
        int need = 0;
        for (int kb = 0; kb < m; kb += kWave) {
            const int mb = min(kWave, m - kb);
            int n_own = 0;  // lane a: partners of key kb + a so far
            const bool staged = mb * cap <= kStage;  // uniform
            if (staged) {
                int open = 0;  // no stencil cell open before the first candidate
                if (wrap) {
                    for (int c0 = 0; c0 < total; c0 += 3 * kWave)
                        list_pass<TPK, true, true, HALF, TL>(d, p, q, qc, cs0, kb, mb, c0, total, start, pre, ekey, cnt, shx,
                                                         shy, shz, n_own, open, stage, mark);
                } else {
                    for (int c0 = 0; c0 < total; c0 += 6 * kWave)
                        list_pass<TPK, false, true, HALF, TL>(d, p, q, qc, cs0, kb, mb, c0, total, start, pre, ekey, cnt, shx,
                                                          shy, shz, n_own, open, stage, mark);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // write-out: item (a, t, c) = chunk c of key a's lane t, 16 bytes; lanes
                // of consecutive keys write consecutive chunks of the list
                const int cpt = cap / TPK / 8;  // chunks per key lane in the buffer
                const int nitem = mb * TPK * cpt;  // <= kStage / 8 (staged)
                // it / (mb * TPK) in FP32: (it + 1/2) / dv lies at least 1/(2 dv) from an
                // integer, far above the rounding error for it < 2^12, dv <= 2^9
                const int dv = mb * TPK;
                const float rdv = 1.0f / (float)dv;
                for (int i0 = 0; i0 < nitem; i0 += kWave) {  // same trip count on every lane
                    const int it = i0 + l;
                    const int c = (int)(((float)it + 0.5f) * rdv), at = it - c * dv;
                    const int a = at / TPK, t = at - a * TPK;
                    const int na = __shfl(n_own, a & 63);  // every lane takes part in the shuffle
                    const int nlane = na > t ? (na - t + TPK - 1) / TPK : 0;
                    if (it < nitem && c * 8 < nlane) {
                        const uint4 v = *reinterpret_cast<const uint4*>(stage + a * cap + t * (cap / TPK) + c * 8);
                        *reinterpret_cast<uint4*>(d.list + list_addr(cs0 + kb + a, 8 * c * TPK + t, TPK, rows)) = v;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else if (wrap) {
                int open = 0;
                for (int c0 = 0; c0 < total; c0 += 3 * kWave)
                    list_pass<TPK, true, false, HALF, TL>(d, p, q, qc, cs0, kb, mb, c0, total, start, pre, ekey, cnt, shx, shy,
                                                      shz, n_own, open, stage, mark);
            } else {
                int open = 0;
                for (int c0 = 0; c0 < total; c0 += 6 * kWave)
                    list_pass<TPK, false, false, HALF, TL>(d, p, q, qc, cs0, kb, mb, c0, total, start, pre, ekey, cnt, shx,
                                                       shy, shz, n_own, open, stage, mark);
            }
            if (l < mb) {
                const int nk = n_own < cap ? n_own : cap;
                d.cnt[cs0 + kb + l] = nk;
                q[cs0 + kb + l].cnt = nk;
            }
            need = max(need, __builtin_amdgcn_readlane(wave_incl_max(l < mb ? n_own : 0), 63));
        }
        if (l == 0) {
            atomicMax(&d.tile_need[t], need);
            if (need > cap) {  // entries were dropped: the step stops here (see halted)
                atomicMax(&d.st[b].need, need);
                atomicOr(d.halt, 1);
            }
        }
    };
    {
        for (int c = xcd_block(blockIdx.x, gridDim.x) * 4 + wv; c < ncells; c += gridDim.x * 4) {
            // tables this kernel does not write, read through the scalar cache
            const int b = ld_const(d.tile_box + c / kTile);
            if (!ld_const(&d.st[b].rebuild)) continue;
            const BoxGeom g = ld_geom(d.geom + b);
            if (c - g.cell_off >= g.ncell) continue;
            cell_body(c, b, g);
        }
    }
}

// ---------------------------------------------------------------- forces

template <int PREC>
struct ShiftT {
    using V = double4;  // FP64: periodic image r * L subtracted from q_j - q_i
};
template <>
struct ShiftT<MD_PREC_FP32_MIXED> {
    using V = int4;  // FP32-mixed: stencil offset o * 2^28 added to u_j - u_i
};

// Compensated FP32 accumulation (Kahan): s + c tracks the running sum.
__device__ __forceinline__ void kahan_add(float& s, float& c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Velocity-Verlet pieces on one key, FP64, no contraction (matches the CPU).
__device__ __forceinline__ double kick(double v, double h, double f) {
#pragma clang fp contract(off)
    return v + h * f;
}
__device__ __forceinline__ double scale(double v, double s) {
#pragma clang fp contract(off)
    return v * s;
}
__device__ __forceinline__ double drift(double x, double dt, double v) {
#pragma clang fp contract(off)
    return x + dt * v;
}
__device__ __forceinline__ double norm2(double x, double y, double z) {
#pragma clang fp contract(off)
    return x * x + y * y + z * z;
}

// Striped per-box maximum: each wavefront folds its value into one of kStripes
// cache-line-separated slots, so no single address sees more than a few hundred
// atomics per step.  k_dutc reduces and clears the stripes.
__device__ __forceinline__ void stripe_put(unsigned long long* base, int b, int w, double v) {
    atomicMax(base + ((size_t)b * kStripes + (w & (kStripes - 1))) * kStripeStride,
              (unsigned long long)__double_as_longlong(v));
}

// The end of a force pass for one key: reduce the lanes of a key, then store F,
// or kick (closing half kick; mid-step: closing and opening kicks, drift and the
// fixed-point re-encoding), DUTC maximum and energy partials per wavefront.
template <int PREC, int MODE, int TPK, bool ENERGY, bool HALF>
__device__ __forceinline__ void force_finish(const Dev& d, const Params& p, const BoxGeom& g, int b, int lw, int key,
                                             bool owner, const Pos& qi, uint32_t cc, int sq, int sp, double Fx,
                                             double Fy, double Fz, double pe, double vir, bool f_done = false) {
    const int l = lane_id();
    if (TPK > 1) {
#pragma unroll
        for (int o = 1; o < TPK; o <<= 1) {
            Fx += __shfl_xor(Fx, o);
            Fy += __shfl_xor(Fy, o);
            Fz += __shfl_xor(Fz, o);
            if (ENERGY) {
                pe += __shfl_xor(pe, o);
                vir += __shfl_xor(vir, o);
            }
        }
    }
    if (HALF) {  // each pair once: its energy and virial count twice against the full list's halves
        pe *= 2.0;
        vir *= 2.0;
    }
    double ke = 0.0, w2 = 0.0, m2 = 0.0;
    if (MODE == kForceOnly) {
        if (owner && HALF) {  // other keys add their reactions to this particle concurrently
            if (!f_done) {  // else already added through the wavefront's LDS accumulators
                unsafeAtomicAdd(d.fx + key, Fx);
                unsafeAtomicAdd(d.fy + key, Fy);
                unsafeAtomicAdd(d.fz + key, Fz);
            }
        } else if (owner) {
            d.fx[key] = Fx;
            d.fy[key] = Fy;
            d.fz[key] = Fz;
        }
        if (owner) {
            if (ENERGY) ke = 0.5 * p.mass * norm2(d.vx[sp][key], d.vy[sp][key], d.vz[sp][key]);
        }
    } else if (MODE == kForceEnd) {
        if (owner) {
            const double vx = kick(d.vx[sp][key], p.h, Fx);
            const double vy = kick(d.vy[sp][key], p.h, Fy);
            const double vz = kick(d.vz[sp][key], p.h, Fz);
            d.vx[sp][key] = vx;
            d.vy[sp][key] = vy;
            d.vz[sp][key] = vz;
            d.fx[key] = Fx;
            d.fy[key] = Fy;
            d.fz[key] = Fz;
            if (ENERGY) ke = 0.5 * p.mass * norm2(vx, vy, vz);
        }
    } else {  // kForceMid
        if (owner) {
            double vx = kick(kick(ld_stream(d.vx[sp] + key), p.h, Fx), p.h, Fx);
            double vy = kick(kick(ld_stream(d.vy[sp] + key), p.h, Fy), p.h, Fy);
            double vz = kick(kick(ld_stream(d.vz[sp] + key), p.h, Fz), p.h, Fz);
            st_stream(d.vx[sp] + key, vx);
            st_stream(d.vy[sp] + key, vy);
            st_stream(d.vz[sp] + key, vz);
            const Pos xn = make_pos(drift(qi.x, p.dt, vx), drift(qi.y, p.dt, vy), drift(qi.z, p.dt, vz), qi.cc,
                                    qi.cnt);
            d.q[sq ^ 1][key] = xn;
            if (PREC == MD_PREC_FP32_MIXED) put_u(d.u[sq ^ 1], key, units3(xn, cc, g));
            w2 = norm2(vx, vy, vz);
            if (d.qb) {
                const double4 xb = d.qb[key];
                m2 = norm2(xn.x - xb.x, xn.y - xb.y, xn.z - xb.z);
            }
        }
    }
    if (MODE == kForceMid) {
        const double wm = wave_max(w2);
        if (l == 0) stripe_put(d.vmax_s, b, lw, wm);
        if (d.qb) {
            const double mm = wave_max(m2);
            if (l == 0) stripe_put(d.disp_s, b, lw, mm);
        }
    }
    if (ENERGY) {
        const double ks = wave_sum(ke);
        const double ps = wave_sum(owner ? pe : 0.0);
        const double vs = wave_sum(owner ? vir : 0.0);
        if (l == 0) {
            d.ke_part[lw] = ks;
            d.pe_part[lw] = ps;
            d.vir_part[lw] = vs;
        }
    }
}

// Algorithm 1 on the GPU.  PREC: MD_PREC_FP64 or MD_PREC_FP32_MIXED.
// MODE: kForceOnly / kForceEnd / kForceMid.  ENERGY: per-wave KE and PE partials.
// Each lane reads 8 list entries per 16-byte load and keeps 8 partner gathers in
// flight (Algorithm 1's unrolling for latency hiding, in GPU form).  A list
// entry names a stencil cell and a rank in it; the wavefront first tabulates, in
// LDS, the 27 stencil cells of each distinct cell its keys live in: FP64 keeps
// the start slot and the periodic image code, FP32-mixed the start slot and the
// fixed-point stencil offset (one 16-byte record).  The cutoff test is a select,
// not a branch (as Algorithm 1's mask w), and only a lane's last, partial chunk
// of entries pays for an end-of-list check.
constexpr int kHomeMax = 12;  // distinct key cells per wavefront served from LDS
constexpr int kAccCap = 512;  // half list: partner accumulators per wavefront in LDS

// Record of stencil cell s of the cell with packed coordinates cc: its start slot
// and the periodic image code of the partners in it (start | code << 27).
__device__ __forceinline__ uint32_t force_rec(const Dev& d, uint32_t cc, int s, const BoxGeom& g) {
    uint32_t img;
    const int nc = stencil_cell(cc, s, g, &img);
    return (uint32_t)d.cell_start[nc] | (img << kIdxBits);
}

// HALF (half list, kForceOnly, one lane per key): the reaction -f d of every pair
// goes to the partner by an atomic add, and the key's own sum is added likewise;
// F must be zero before the pass.
template <int PREC, int MODE, int TPK, bool ENERGY, bool HALF = false>
__global__ __launch_bounds__(kBlock) void k_force(Dev d, Params p) {
    if (halted(d)) return;
    static_assert(!HALF || (MODE == kForceOnly && TPK == 1), "half lists: forces only, one lane per key");
    constexpr int K = kWave / TPK;
    constexpr int U = 8;  // entries per iteration (one 16-byte chunk)
    constexpr bool MIX = PREC == MD_PREC_FP32_MIXED;
    using Rec = uint32_t;
    // FP64: image term per code, one 27-entry array per axis (8-byte words read by code)
    __shared__ double shift[MIX ? 1 : kBlock / kWave][3 * 27];
    __shared__ uint32_t home_cc[kBlock / kWave][kWave];
    __shared__ Rec tab[kBlock / kWave][kHomeMax * 27];
    // FP32-mixed: image term -r * n * uoff (modulo 2^32) of image code r, one array per
    // axis: 4-byte words read by code, so lanes spread over the banks (or share a word)
    __shared__ int32_t soff[MIX ? kBlock / kWave : 1][MIX ? 3 * 27 : 1];
    const int l = lane_id(), wib = wave_in_block(), sub = l % TPK;
    const int lw = xcd_block(blockIdx.x, gridDim.x) * 4 + wib;
    const int nlw = p.nwave * TPK;
    const bool wave_ok = lw < nlw;
    const int b = wave_ok ? ld_const(d.wave_box + ((lw * K) >> 6)) : 0;
    if constexpr (!MIX) {
        if (l < 27) {
            const double4 sh = d.dshift[b * 27 + l];
            shift[wib][l] = sh.x;
            shift[wib][27 + l] = sh.y;
            shift[wib][54 + l] = sh.z;
        }
    } else {
        if (l < 27) {
            const BoxGeom& gb = d.geom[b];
            soff[wib][l] = img_units(l % 3 - 1, gb.n[0], gb.uoff[0]);
            soff[wib][27 + l] = img_units((l / 3) % 3 - 1, gb.n[1], gb.uoff[1]);
            soff[wib][54 + l] = img_units(l / 9 - 1, gb.n[2], gb.uoff[2]);
        }
    }
    __syncthreads();
    if (!wave_ok) return;

    const BoxGeom& g = d.geom[b];  // b is uniform: scalar loads
    const int sq = d.st[b].sq, sp = d.st[b].sp;
    const int key = lw * K + l / TPK;
    const bool active = key - g.slot_off < g.npart;
    const Pos qi = d.q[sq][active ? key : g.slot_off];
    const uint32_t cc = active ? qi.cc : 0xffffffffu;

    // distinct cells of this wavefront's keys (keys are sorted by cell)
    const uint32_t cprev = __shfl_up(cc, TPK);
    const bool head = active && sub == 0 && (l < TPK || cprev != cc);
    const unsigned long long hm = __ballot(head);
    const int nhome = __popcll(hm);
    const int h = __popcll(hm & (l == 63 ? ~0ull : ((2ull << l) - 1ull))) - 1;
    const bool tabled = nhome <= kHomeMax;  // uniform
    if (tabled) {
        if (head) home_cc[wib][h] = cc;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int idx = l; idx < nhome * 27; idx += kWave) {
            const int hh = idx / 27;
            tab[wib][idx] = force_rec(d, home_cc[wib][hh], idx - hh * 27, g);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // Half list: the reactions of a wavefront whose keys lie in one row of cells,
    // away from the x faces, accumulate in LDS.  Its forward partners then lie in
    // five row segments -- the same row from the first home cell, and rows
    // (dy, dz) = (1, 0), (-1, 1), (0, 1), (1, 1) from one cell before it, each up to
    // one cell past the last home cell -- every one a contiguous run of slots.  The
    // accumulators leave once, as atomic adds to consecutive slots; other wavefronts
    // add every reaction to HBM directly.
    using Acc = std::conditional_t<MIX, float, double>;
    __shared__ Acc acc[HALF ? kBlock / kWave : 1][HALF ? 3 * kAccCap : 1];
    __shared__ int32_t atab[HALF ? kBlock / kWave : 1][HALF ? kHomeMax * 27 : 1];
    __shared__ int32_t segs[HALF ? kBlock / kWave : 1][10];  // first slot, then LDS base, of each row segment
    bool local = false;
    int ntot = 0;
    if constexpr (HALF) {
        if (tabled) {
            const uint32_t c0 = home_cc[wib][0], c1 = home_cc[wib][nhome - 1];
            const int x0 = (int)(c0 & 1023), x1 = (int)(c1 & 1023);
            local = (c0 >> 10) == (c1 >> 10) && x0 >= 1 && x1 <= g.n[0] - 2;
        }
        if (local) {
            const uint32_t c0 = home_cc[wib][0], c1 = home_cc[wib][nhome - 1];
            const int x0 = (int)(c0 & 1023), x1 = (int)(c1 & 1023);
            int lo = 0, len = 0;
            if (l < 5) {  // row segment l: (dy, dz) = (0,0), (1,0), (-1,1), (0,1), (1,1)
                const int oy = l == 0 ? 0 : (l == 1 ? 1 : l - 3), oz = l < 2 ? 0 : 1;
                int y = (int)((c0 >> 10) & 1023) + oy, z = (int)(c0 >> 20) + oz;
                if (y < 0) y += g.n[1];
                if (y >= g.n[1]) y -= g.n[1];
                if (z >= g.n[2]) z -= g.n[2];
                const int row = g.cell_off + (z * g.n[1] + y) * g.n[0];
                const int ca = row + (l == 0 ? x0 : x0 - 1), cb = row + x1 + 1;
                lo = d.cell_start[ca];
                len = d.cell_start[cb] + d.cell_cnt[cb] - lo;
            }
            const int incl = wave_incl_scan(len);
            ntot = __builtin_amdgcn_readlane(incl, 4);
            local = ntot <= kAccCap;  // uniform
            if (local) {
                if (l < 5) {
                    segs[wib][l] = lo;
                    segs[wib][5 + l] = incl - len;
                }
                for (int i = l; i < 3 * ntot; i += kWave) acc[wib][i] = Acc(0);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int idx = l; idx < nhome * 27; idx += kWave) {
                    const int hh = idx / 27, s = idx - hh * 27;
                    int v = -1;  // backward cells hold no half-list partners
                    if (s >= 13) {
                        uint32_t img;
                        const int nc = stencil_cell(home_cc[wib][hh], s, g, &img);
                        const int r = s <= 14 ? 0 : (s - 15) / 3 + 1;
                        v = segs[wib][5 + r] + (d.cell_start[nc] - segs[wib][r]);
                    }
                    atab[wib][idx] = v;
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
    }
    auto lds_add = [&](int li, Acc x, Acc y, Acc z) {
        __hip_atomic_fetch_add(&acc[wib][3 * li], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&acc[wib][3 * li + 1], y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(&acc[wib][3 * li + 2], z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };

    double Fx = 0.0, Fy = 0.0, Fz = 0.0, pe = 0.0, vir = 0.0;  // vir: sum_j f r^2 (energy passes)
    // The pair loop, instantiated twice so the choice between the LDS table and
    // direct lookups is made once per wavefront, outside the loop.
    auto pair_loop = [&](auto tabled_c) {
        constexpr bool TB = decltype(tabled_c)::value;
        const int n_i = qi.cnt;
        const int nl = n_i > sub ? (n_i - sub + TPK - 1) / TPK : 0;  // this lane's entries
        const int nfull = nl >> 3, ntail = nl & 7;
        const uint4* __restrict__ l4 = reinterpret_cast<const uint4*>(d.list + (size_t)lw * p.rows * kWave) + l;
        const Rec* __restrict__ tb = tab[wib] + h * 27;
        auto rec = [&](uint32_t s) -> Rec {
            if constexpr (TB)
                return tb[s];
            else
                return force_rec(d, cc, (int)s, g);
        };
        // entry k of a chunk: stencil cell and rank (8 entries in 4 words)
        auto ent_s = [](const uint4& raw, int k) -> uint32_t {
            const uint32_t w = k < 2 ? raw.x : k < 4 ? raw.y : k < 6 ? raw.z : raw.w;
            return (k & 1) ? w >> 27 : (w >> kOffBits) & 31u;
        };
        auto ent_r = [](const uint4& raw, int k) -> uint32_t {
            const uint32_t w = k < 2 ? raw.x : k < 4 ? raw.y : k < 6 ? raw.z : raw.w;
            return (k & 1) ? (w >> 16) & (kMaxCellCount - 1) : w & (kMaxCellCount - 1);
        };
        uint4 raw_next = nl > 0 ? ld_stream(l4) : make_uint4(0u, 0u, 0u, 0u);
        if constexpr (!MIX) {
            const Pos* __restrict__ q = d.q[sq];
            const double rc2 = p.rc2, c2x8 = 8.0 * p.c2;
            const bool fast = p.fastrcp != 0;  // uniform
            // CHK: the lane's last chunk, entries from `valid` on are padding
            auto chunk = [&](int c, auto chk_c, int valid) {
                constexpr bool CHK = decltype(chk_c)::value;
                const uint4 raw = raw_next;
                uint32_t js[U], img[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const bool ok = !CHK || k < valid;
                    const uint32_t t = rec(ok ? ent_s(raw, k) : 13u);
                    js[k] = ok ? (t & kIdxMask) + ent_r(raw, k) : (uint32_t)key;
                    img[k] = ok ? t >> kIdxBits : 13u;
                }
                Pos qj[U];
#pragma unroll
                for (int k = 0; k < U; ++k)  // 32-bit byte offsets: slots < 2^27
                    qj[k] = *reinterpret_cast<const Pos*>(reinterpret_cast<const char*>(q) + (js[k] << 5));
                // next chunk's entries, issued after the gathers: the load counter
                // retires in order, so this load does not delay them
                if (!CHK && (c + 1 < nfull || ntail)) raw_next = ld_stream(l4 + (size_t)(c + 1) * kWave);
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const double* __restrict__ sh = shift[wib] + img[k];
                    const double dx = (qj[k].x - qi.x) - sh[0];
                    const double dy = (qj[k].y - qi.y) - sh[27];
                    const double dz = (qj[k].z - qi.z) - sh[54];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const bool in = (!CHK || k < valid) && r2 < rc2;
                    double f, e = 0.0;
                    if (fast) {
                        // Sec. III.C: with xt ~ 1/r^2 and t = xt r^2 = 1 + eps,
                        // r^-2n = xt^n ((n + 1) - n t) + O(eps^2)
                        const double xt = __builtin_amdgcn_rcp(r2);
                        const double t = xt * r2;
                        const double x2 = xt * xt, x3 = x2 * xt, x4 = x2 * x2;
                        const double r8 = x4 * (5.0 - 4.0 * t), r14 = x4 * x3 * (8.0 - 7.0 * t);
                        f = in ? 24.0 * r8 - 48.0 * r14 + c2x8 : 0.0;
                        if (ENERGY) e = x3 * x3 * (7.0 - 6.0 * t) - x3 * (4.0 - 3.0 * t);
                    } else {
                        const double inv = 1.0 / r2;
                        const double inv3 = inv * inv * inv;
                        f = in ? (24.0 * inv3 - 48.0 * inv3 * inv3) * inv + c2x8 : 0.0;
                        if (ENERGY) e = inv3 * inv3 - inv3;
                    }
                    Fx += f * dx;
                    Fy += f * dy;
                    Fz += f * dz;
                    if (HALF && in) {  // Newton's third law: the reaction on the partner
                        if (local) {
                            lds_add(atab[wib][h * 27 + (int)ent_s(raw, k)] + (int)ent_r(raw, k), -(f * dx), -(f * dy),
                                    -(f * dz));
                        } else {
                            unsafeAtomicAdd(d.fx + js[k], -(f * dx));
                            unsafeAtomicAdd(d.fy + js[k], -(f * dy));
                            unsafeAtomicAdd(d.fz + js[k], -(f * dz));
                        }
                    }
                    if (ENERGY) {
                        pe += in ? 2.0 * (e + p.c2 * r2 + p.c0) : 0.0;
                        vir += in ? f * r2 : 0.0;
                    }
                }
            };
            for (int c = 0; c < nfull; ++c) chunk(c, std::false_type{}, U);
            if (ntail) chunk(nfull, std::true_type{}, ntail);
        } else {
            const int32_t* __restrict__ u = d.u[sq];
            const int4 ui = units3(qi, cc, g);  // own coordinate from the record: no extra load
            // lengths stay in fixed-point units: r^2 in units^2, 1/r^2 rescaled once
            const float rc2u = g.rc2u, lam2inv = g.lam2inv, lam2 = g.lam * g.lam, c2x8 = 8.0f * p.c2f;
            const float irc2 = p.irc2f;
            // the clamp serves full lists only: a half list's reactions go to partners directly
            const bool clampf = p.clamp != 0 && !HALF;
            const double lamd = (double)g.lam;
            float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f, pes = 0.f, virs = 0.f;
            auto chunk = [&](int c, auto chk_c, int valid) {
                constexpr bool CHK = decltype(chk_c)::value;
                const uint4 raw = raw_next;
                uint32_t st[U], js[U], img[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const bool ok = !CHK || k < valid;
                    st[k] = ok ? ent_s(raw, k) : 13u;
                    const uint32_t t = rec(st[k]);
                    js[k] = ok ? (t & kIdxMask) + ent_r(raw, k) : (uint32_t)key;
                    img[k] = ok ? t >> kIdxBits : 13u;
                }
                int4 uj[U];
#pragma unroll
                for (int k = 0; k < U; ++k)  // 32-bit byte offsets: slots < 2^27
                {  // 32-bit byte offsets from a uniform base: slots < 2^27, 12 bytes each
                    const U3 t = *reinterpret_cast<const U3*>(reinterpret_cast<const char*>(u) + js[k] * 12u);
                    uj[k] = make_int4(t.x, t.y, t.z, 0);
                }
                if (!CHK && (c + 1 < nfull || ntail)) raw_next = ld_stream(l4 + (size_t)(c + 1) * kWave);
                // the stencil offsets are read again below rather than held across the gathers
                __builtin_amdgcn_sched_barrier(0);
                float bx = 0.f, by = 0.f, bz = 0.f;  // plain FP32 sum of this batch
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const int* __restrict__ so = soff[wib] + img[k];
                    // exact integer separation in units (modulo 2^32, far inside int32),
                    // one rounding to FP32
                    const float dx = (float)(int)((uint32_t)uj[k].x + (uint32_t)so[0] - (uint32_t)ui.x);
                    const float dy = (float)(int)((uint32_t)uj[k].y + (uint32_t)so[27] - (uint32_t)ui.y);
                    const float dz = (float)(int)((uint32_t)uj[k].z + (uint32_t)so[54] - (uint32_t)ui.z);
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const bool in = (!CHK || k < valid) && r2 < rc2u;
                    const float inv0 = __builtin_amdgcn_rcpf(r2) * lam2inv;  // 1/r^2 in length units
                    // Eq. 1 (f(rc) = 0): entries beyond rc evaluated at rc, as the row-tile pass does
                    const float inv = clampf ? fmaxf(inv0, irc2) : inv0;
                    const float inv3 = inv * inv * inv;
                    const float fv = (inv3 * inv) * (24.0f - 48.0f * inv3) + c2x8;
                    const float f = (clampf ? (!CHK || k < valid) : in) ? fv : 0.0f;
                    const float fdx = f * dx, fdy = f * dy, fdz = f * dz;
                    bx += fdx;
                    by += fdy;
                    bz += fdz;
                    if (HALF && in) {  // Newton's third law: the reaction on the partner, in lengths
                        if (local) {
                            const float lamf = g.lam;  // a power of two: exact scaling
                            lds_add(atab[wib][h * 27 + (int)st[k]] + (int)ent_r(raw, k), -(fdx * lamf), -(fdy * lamf),
                                    -(fdz * lamf));
                        } else {
                            unsafeAtomicAdd(d.fx + js[k], -(double)fdx * lamd);
                            unsafeAtomicAdd(d.fy + js[k], -(double)fdy * lamd);
                            unsafeAtomicAdd(d.fz + js[k], -(double)fdz * lamd);
                        }
                    }
                    if (ENERGY) {
                        const float i3 = inv0 * inv0 * inv0;
                        pes += in ? 2.0f * (i3 * i3 - i3 + p.c2f * (r2 * lam2) + p.c0f) : 0.0f;
                        virs += in ? f * r2 : 0.0f;  // units^2: times lam^2 below
                    }
                }
                kahan_add(sx, cx, bx);  // compensated across batches
                kahan_add(sy, cy, by);
                kahan_add(sz, cz, bz);
            };
            for (int c = 0; c < nfull; ++c) chunk(c, std::false_type{}, U);
            if (ntail) chunk(nfull, std::true_type{}, ntail);
            const double lam = (double)g.lam;  // units back to lengths (a power of two)
            Fx = ((double)sx - (double)cx) * lam;
            Fy = ((double)sy - (double)cy) * lam;
            Fz = ((double)sz - (double)cz) * lam;
            pe = (double)pes;
            vir = (double)virs * lam * lam;
        }
    };
    if (active) {
        if (tabled)
            pair_loop(std::true_type{});
        else
            pair_loop(std::false_type{});
    }
    bool f_done = false;
    if constexpr (HALF) {
        if (local) {  // own sums join the accumulators, which then leave in one pass
            if (active) lds_add(segs[wib][5] + (key - segs[wib][0]), (Acc)Fx, (Acc)Fy, (Acc)Fz);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int i = l; i < ntot; i += kWave) {
                int r = 0;
#pragma unroll
                for (int rr = 1; rr < 5; ++rr) r = i >= segs[wib][5 + rr] ? rr : r;
                const int slot = segs[wib][r] + (i - segs[wib][5 + r]);
                const double ax = (double)acc[wib][3 * i], ay = (double)acc[wib][3 * i + 1],
                             az = (double)acc[wib][3 * i + 2];
                if (ax != 0.0 || ay != 0.0 || az != 0.0) {
                    unsafeAtomicAdd(d.fx + slot, ax);
                    unsafeAtomicAdd(d.fy + slot, ay);
                    unsafeAtomicAdd(d.fz + slot, az);
                }
            }
            f_done = true;
        }
    }
    force_finish<PREC, MODE, TPK, ENERGY, HALF>(d, p, g, b, lw, key, active && sub == 0, qi, cc, sq, sp, Fx, Fy, Fz,
                                                pe, vir, f_done);
}

// FP32-mixed pair forces from a row tile staged in LDS (row-tile list format, one
// lane per key).  A block takes a row tile: wavefront 0 works out the 27 pieces of
// its staged region, the block copies them from the fixed-point array into LDS as
// 16-byte records (coalesced runs of slots; the pieces' image terms added, so every
// record is in the unwrapped frame of the home row), then each lane walks one key's
// list, whose entries are the records' LDS byte offsets.  A pair separation is one
// integer subtraction per axis (exact, modulo 2^32) and one conversion to FP32; the
// arithmetic after that, and the summation order, are those of the gather kernel,
// so both give the same forces bit for bit.  The integration (kicks, drift,
// fixed-point re-encoding, DUTC maximum) follows in the same pass; energy partials
// are summed per tile in a fixed order.  A tile whose region exceeds scap is
// skipped (its build has stopped the step; the host switches to the gather format
// and goes on from that build).
// CLAMP (the Eq. 1 cutoff, whose f(rc) is 0): a list entry beyond rc is evaluated at
// rc instead of being masked, 1/r^2 = max(1/r^2, 1/rc^2) (one instruction for a
// compare and a select); f(rc) rounds to a few 1e-9 in FP32.
template <int MODE, bool ENERGY, bool CLAMP>
__global__ __launch_bounds__(kRtBlock) void k_force_t(Dev d, Params p) {
    if (halted(d)) return;
    constexpr int NW = kRtBlock / kWave;  // wavefronts per block
    constexpr int U = 8;       // entries per 16-byte list chunk
    constexpr int kPc = 27;    // pieces of a staged region
    constexpr int kCopy = 4;   // copy chunks per wavefront in flight
    extern __shared__ U3 stg[];  // p.scap records of 12 bytes
    __shared__ double red[3][NW];
    const int l = lane_id(), wib = wave_in_block();
    const int ntl = ld_const(d.ntiles);
    for (int t = xcd_block(blockIdx.x, gridDim.x); t < ntl; t += gridDim.x) {
        // Staging runs at a raised wavefront priority, the pair loop at the normal one: a
        // block that starts a tile gets its loads issued ahead of the arithmetic of the
        // CU's other blocks, so their pair loops cover its memory latency.
        __builtin_amdgcn_s_setprio(2);
        const int4 tr = d.rtile[t];
        const int b = __builtin_amdgcn_readfirstlane(tr.x);
        const BoxGeom g = ld_geom(d.geom + b);
        const int lr = __builtin_amdgcn_readfirstlane(tr.y), xa = __builtin_amdgcn_readfirstlane(tr.z),
                  xb = __builtin_amdgcn_readfirstlane(tr.w);
        const int cz = gdiv(g, lr, 1), cy = lr - cz * g.n[1];
        const int sq = ld_const(&d.st[b].sq), sp = ld_const(&d.st[b].sp);
        // every wavefront works out the pieces itself (lane p holds piece p): no barrier
        int ps0 = 0, plen = 0, pox = 0, poy = 0, poz = 0;
        if (l < kPc) tile_piece(d, g, cy, cz, xa, xb, l, ps0, plen, pox, poy, poz);
        const int pincl = wave_incl_sum(plen);
        const int S = __builtin_amdgcn_readlane(pincl, kPc - 1);
        // keys: the home cells [xa, xb) of the home row (inside piece 13)
        const int rowc = g.cell_off + (cz * g.n[1] + cy) * g.n[0];
        const int k0 = ld_const(d.cell_start + rowc + xa);
        const int k1 = ld_const(d.cell_start + rowc + xb - 1) + ld_const(d.cell_cnt + rowc + xb - 1);
        if (S > p.scap) continue;  // uniform over the block; nothing staged yet
        // this thread's first key: its record, velocity and first two list chunks, fetched
        // while the block stages (a list holds at least 8 entries per lane, 16 when rows >= 16)
        int kb = k0;
        int key = kb + (int)threadIdx.x;
        bool active = key < k1;
        int ks = active ? key : k0;
        Pos qi = d.q[sq][ks];
        double v0x = ld_stream(d.vx[sp] + ks), v0y = ld_stream(d.vy[sp] + ks), v0z = ld_stream(d.vz[sp] + ks);
        const uint4* __restrict__ l4 = reinterpret_cast<const uint4*>(d.list) + (size_t)(ks >> 6) * p.rows * 8 + (ks & 63);
        uint4 raw_a = ld_stream(l4);
        uint4 raw_b = p.rows >= 16 ? ld_stream(l4 + kWave) : make_uint4(0u, 0u, 0u, 0u);
        // stage: 64-record chunk c of the pieces goes to wavefront c % NW; the chunk's
        // piece is the number of pieces whose chunks all lie before it.  Per piece p
        // (first chunk cs): record c * 64 + l of the pieces' chunk space comes from slot
        // src_p + c * 64 + l and goes to dst_p + c * 64 + l while c * 64 + l < end_p.
        {
            const int pch = (plen + kWave - 1) >> 6;  // 64-record copy chunks of piece l
            const int chincl = wave_incl_sum(pch);
            const int NC = __builtin_amdgcn_readlane(chincl, kPc - 1);
            const int cs = chincl - pch;
            const int src = ps0 - kWave * cs, dst = (pincl - plen) - kWave * cs, end = plen + kWave * cs;
            const int32_t* __restrict__ u = d.u[sq];
            for (int c0 = wib; c0 < NC; c0 += NW * kCopy) {
                U3 v[kCopy];
                int at[kCopy], ox[kCopy], oy[kCopy], oz[kCopy];
#pragma unroll
                for (int k = 0; k < kCopy; ++k) {
                    const int c = c0 + NW * k;
                    at[k] = -1;
                    if (c < NC) {  // uniform
                        const int pc = __popcll(__ballot(l < kPc && chincl <= c));
                        const int i = c * kWave + l;
                        ox[k] = __builtin_amdgcn_readlane(pox, pc);
                        oy[k] = __builtin_amdgcn_readlane(poy, pc);
                        oz[k] = __builtin_amdgcn_readlane(poz, pc);
                        if (i < __builtin_amdgcn_readlane(end, pc)) {
                            v[k] = *reinterpret_cast<const U3*>(u + 3 * (__builtin_amdgcn_readlane(src, pc) + i));
                            at[k] = __builtin_amdgcn_readlane(dst, pc) + i;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < kCopy; ++k)
                    if (at[k] >= 0)
                        stg[at[k]] = U3{(int)((uint32_t)v[k].x + (uint32_t)ox[k]), (int)((uint32_t)v[k].y + (uint32_t)oy[k]),
                                        (int)((uint32_t)v[k].z + (uint32_t)oz[k])};
            }
        }
        __syncthreads();
        const float rc2u = g.rc2u, lam2inv = g.lam2inv, lam2 = g.lam * g.lam, c2x8 = 8.0f * p.c2f;
        const float irc2 = p.irc2f;  // 1 / rc^2 in length units (FP32)
        const double lam = (double)g.lam;  // units back to lengths (a power of two)
        const char* __restrict__ sb = reinterpret_cast<const char*>(stg);
        double e_ke = 0.0, e_pe = 0.0, e_vir = 0.0;
        for (;;) {  // rounds of kRtBlock keys: a one-cell tile may hold more (uniform)
            __builtin_amdgcn_s_setprio(0);  // the pair loop at the normal priority
            const uint32_t cc = qi.cc;
            const int4 ui = units3(qi, cc, g);  // own coordinate, from the record: no extra load
            const uint32_t kx = (uint32_t)ui.x, ky = (uint32_t)ui.y, kz = (uint32_t)ui.z;
            const int nl = active ? qi.cnt : 0;
            const int nfull = nl >> 3, ntail = nl & 7;
            float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy2 = 0.f, cz2 = 0.f, pes = 0.f, virs = 0.f;
            // list chunks two ahead: the next chunk's load has a whole chunk of math to land
            auto chunk = [&](int c, auto chk_c, int valid) {
                constexpr bool CHK = decltype(chk_c)::value;
                const uint4 raw = raw_a;
                U3 rj[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const uint32_t w = k < 2 ? raw.x : k < 4 ? raw.y : k < 6 ? raw.z : raw.w;
                    uint32_t off = (k & 1) ? w >> 16 : w & 0xffffu;
                    if (CHK && k >= valid) off = 0u;  // padding entries: any record, masked below
                    rj[k] = *reinterpret_cast<const U3*>(sb + off);
                }
                if (!CHK) {
                    raw_a = raw_b;
                    if (8 * (c + 2) < nl) raw_b = ld_stream(l4 + (size_t)(c + 2) * kWave);
                }
                float bx = 0.f, by = 0.f, bz = 0.f;  // plain FP32 sum of this batch
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    // exact integer separation in units, one rounding to FP32
                    const float dx = (float)(int)((uint32_t)rj[k].x - kx);
                    const float dy = (float)(int)((uint32_t)rj[k].y - ky);
                    const float dz = (float)(int)((uint32_t)rj[k].z - kz);
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const bool in = (!CHK || k < valid) && r2 < rc2u;
                    const float inv0 = __builtin_amdgcn_rcpf(r2) * lam2inv;  // 1/r^2 in length units
                    const float inv = CLAMP ? fmaxf(inv0, irc2) : inv0;
                    const float inv3 = inv * inv * inv;
                    const float fv = (inv3 * inv) * (24.0f - 48.0f * inv3) + c2x8;
                    const float f = CLAMP && !CHK ? fv : (in || (CLAMP && k < valid) ? fv : 0.0f);
                    bx += f * dx;
                    by += f * dy;
                    bz += f * dz;
                    if (ENERGY) {
                        const float i3 = inv0 * inv0 * inv0;
                        pes += in ? 2.0f * (i3 * i3 - i3 + p.c2f * (r2 * lam2) + p.c0f) : 0.0f;
                        virs += in ? f * r2 : 0.0f;  // units^2: times lam^2 below
                    }
                }
                kahan_add(sx, cx, bx);  // compensated across batches
                kahan_add(sy, cy2, by);
                kahan_add(sz, cz2, bz);
            };
            for (int c = 0; c < nfull; ++c) chunk(c, std::false_type{}, U);
            if (ntail) chunk(nfull, std::true_type{}, ntail);
            __builtin_amdgcn_s_setprio(1);  // the epilogue's loads and stores ahead of pair loops
            const double Fx = ((double)sx - (double)cx) * lam;
            const double Fy = ((double)sy - (double)cy2) * lam;
            const double Fz = ((double)sz - (double)cz2) * lam;
            double ke = 0.0, w2 = 0.0, m2 = 0.0;
            if (active) {
                if (MODE == kForceOnly) {
                    d.fx[key] = Fx;
                    d.fy[key] = Fy;
                    d.fz[key] = Fz;
                    if (ENERGY) ke = 0.5 * p.mass * norm2(v0x, v0y, v0z);
                } else if (MODE == kForceEnd) {
                    const double vx = kick(v0x, p.h, Fx);
                    const double vy = kick(v0y, p.h, Fy);
                    const double vz = kick(v0z, p.h, Fz);
                    d.vx[sp][key] = vx;
                    d.vy[sp][key] = vy;
                    d.vz[sp][key] = vz;
                    d.fx[key] = Fx;
                    d.fy[key] = Fy;
                    d.fz[key] = Fz;
                    if (ENERGY) ke = 0.5 * p.mass * norm2(vx, vy, vz);
                } else {  // kForceMid: close step n, open step n+1, drift, re-encode
                    const double vx = kick(kick(v0x, p.h, Fx), p.h, Fx);
                    const double vy = kick(kick(v0y, p.h, Fy), p.h, Fy);
                    const double vz = kick(kick(v0z, p.h, Fz), p.h, Fz);
                    st_stream(d.vx[sp] + key, vx);
                    st_stream(d.vy[sp] + key, vy);
                    st_stream(d.vz[sp] + key, vz);
                    const Pos xn = make_pos(drift(qi.x, p.dt, vx), drift(qi.y, p.dt, vy), drift(qi.z, p.dt, vz), cc,
                                            qi.cnt);
                    d.q[sq ^ 1][key] = xn;
                    put_u(d.u[sq ^ 1], key, units3(xn, cc, g));
                    w2 = norm2(vx, vy, vz);
                    if (d.qb) {
                        const double4 xbq = d.qb[key];
                        m2 = norm2(xn.x - xbq.x, xn.y - xbq.y, xn.z - xbq.z);
                    }
                }
            }
            if (MODE == kForceMid) {
                const double wm = wave_max(w2);
                if (l == 0) stripe_put(d.vmax_s, b, t * 4 + wib, wm);
                if (d.qb) {
                    const double mm = wave_max(m2);
                    if (l == 0) stripe_put(d.disp_s, b, t * 4 + wib, mm);
                }
            }
            if (ENERGY && active) {
                e_ke += ke;
                e_pe += (double)pes;
                e_vir += (double)virs * lam * lam;
            }
            kb += kRtBlock;
            if (kb >= k1) break;
            key = kb + (int)threadIdx.x;
            active = key < k1;
            ks = active ? key : k0;
            qi = d.q[sq][ks];
            v0x = ld_stream(d.vx[sp] + ks);
            v0y = ld_stream(d.vy[sp] + ks);
            v0z = ld_stream(d.vz[sp] + ks);
            l4 = reinterpret_cast<const uint4*>(d.list) + (size_t)(ks >> 6) * p.rows * 8 + (ks & 63);
            raw_a = ld_stream(l4);
            raw_b = p.rows >= 16 ? ld_stream(l4 + kWave) : make_uint4(0u, 0u, 0u, 0u);
        }
        if (ENERGY) {  // the tile's partials, summed in a fixed order
            const double ks = wave_sum(e_ke), ps = wave_sum(e_pe), vs = wave_sum(e_vir);
            __syncthreads();  // red of the previous tile has been read
            if (l == 0) {
                red[0][wib] = ks;
                red[1][wib] = ps;
                red[2][wib] = vs;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double a0 = red[0][0], a1 = red[1][0], a2 = red[2][0];
                for (int w = 1; w < NW; ++w) {
                    a0 += red[0][w];
                    a1 += red[1][w];
                    a2 += red[2][w];
                }
                d.ke_part[t] = a0;
                d.pe_part[t] = a1;
                d.vir_part[t] = a2;
            }
        }
        __syncthreads();  // the next tile's staging reuses the LDS
    }
}

// FP64 pair forces from a row tile staged in LDS (row-tile list format, one lane per
// key): the tiles, pieces and list entries of k_force_t, with FP64 position records
// (x, y, z; an entry is 24 times the staged index) staged with each piece's periodic
// image added (x - L where the piece wrapped below 0, x + L above), so a separation is
// three FP64 subtractions.  For pairs that do not cross a periodic face that is the
// gather pass's separation bit for bit; across a face the image is added before the
// subtraction instead of after (one rounding of a different sum).  The pair scalar,
// the summation order and the integration are the gather pass's (IEEE division, or
// the hardware reciprocal with the correction of Sec. III.C).
struct D3 {
    double x, y, z;
};
template <int MODE, bool ENERGY>
__global__ __launch_bounds__(kRtBlock) void k_force_t64(Dev d, Params p) {
    if (halted(d)) return;
    constexpr int NW = kRtBlock / kWave;
    constexpr int U = 8, kPc = 27, kCopy = 4;
    extern __shared__ D3 stg64[];  // p.scap records of 24 bytes
    __shared__ double red[3][NW];
    const int l = lane_id(), wib = wave_in_block();
    const int ntl = ld_const(d.ntiles);
    for (int t = xcd_block(blockIdx.x, gridDim.x); t < ntl; t += gridDim.x) {
        __builtin_amdgcn_s_setprio(2);  // staging ahead of pair loops, as in k_force_t
        const int4 tr = d.rtile[t];
        const int b = __builtin_amdgcn_readfirstlane(tr.x);
        const BoxGeom g = ld_geom(d.geom + b);
        const int lr = __builtin_amdgcn_readfirstlane(tr.y), xa = __builtin_amdgcn_readfirstlane(tr.z),
                  xb = __builtin_amdgcn_readfirstlane(tr.w);
        const int cz = gdiv(g, lr, 1), cy = lr - cz * g.n[1];
        const int sq = ld_const(&d.st[b].sq), sp = ld_const(&d.st[b].sp);
        int ps0 = 0, plen = 0, rx = 0, ry = 0, rz = 0;
        if (l < kPc) {
            int ox, oy, oz;
            tile_piece(d, g, cy, cz, xa, xb, l, ps0, plen, ox, oy, oz);
            tile_piece_img(g, cy, cz, l, rx, ry, rz);
        }
        const int pincl = wave_incl_sum(plen);
        const int S = __builtin_amdgcn_readlane(pincl, kPc - 1);
        const int rowc = g.cell_off + (cz * g.n[1] + cy) * g.n[0];
        const int k0 = ld_const(d.cell_start + rowc + xa);
        const int k1 = ld_const(d.cell_start + rowc + xb - 1) + ld_const(d.cell_cnt + rowc + xb - 1);
        if (S > p.scap) continue;  // uniform over the block; nothing staged yet
        int kb = k0;
        int key = kb + (int)threadIdx.x;
        bool active = key < k1;
        int ks = active ? key : k0;
        Pos qi = d.q[sq][ks];
        double v0x = ld_stream(d.vx[sp] + ks), v0y = ld_stream(d.vy[sp] + ks), v0z = ld_stream(d.vz[sp] + ks);
        const uint4* __restrict__ l4 = reinterpret_cast<const uint4*>(d.list) + (size_t)(ks >> 6) * p.rows * 8 + (ks & 63);
        uint4 raw_a = ld_stream(l4);
        uint4 raw_b = p.rows >= 16 ? ld_stream(l4 + kWave) : make_uint4(0u, 0u, 0u, 0u);
        {  // staging, as in k_force_t: 64-record chunks dealt round-robin to the wavefronts
            const int pch = (plen + kWave - 1) >> 6;
            const int chincl = wave_incl_sum(pch);
            const int NC = __builtin_amdgcn_readlane(chincl, kPc - 1);
            const int cs = chincl - pch;
            const int src = ps0 - kWave * cs, dst = (pincl - plen) - kWave * cs, end = plen + kWave * cs;
            const Pos* __restrict__ q = d.q[sq];
            for (int c0 = wib; c0 < NC; c0 += NW * kCopy) {
                D3 v[kCopy];
                int at[kCopy];
#pragma unroll
                for (int k = 0; k < kCopy; ++k) {
                    const int c = c0 + NW * k;
                    at[k] = -1;
                    if (c < NC) {  // uniform
                        const int pc = __popcll(__ballot(l < kPc && chincl <= c));
                        const int i = c * kWave + l;
                        const double sx = (double)__builtin_amdgcn_readlane(rx, pc) * g.L[0];
                        const double sy = (double)__builtin_amdgcn_readlane(ry, pc) * g.L[1];
                        const double sz = (double)__builtin_amdgcn_readlane(rz, pc) * g.L[2];
                        if (i < __builtin_amdgcn_readlane(end, pc)) {
                            const Pos x = q[__builtin_amdgcn_readlane(src, pc) + i];
                            v[k] = D3{x.x + sx, x.y + sy, x.z + sz};
                            at[k] = __builtin_amdgcn_readlane(dst, pc) + i;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < kCopy; ++k)
                    if (at[k] >= 0) stg64[at[k]] = v[k];
            }
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
        const double rc2 = p.rc2, c2x8 = 8.0 * p.c2;
        const bool fast = p.fastrcp != 0;  // uniform
        const char* __restrict__ sb = reinterpret_cast<const char*>(stg64);
        double e_ke = 0.0, e_pe = 0.0, e_vir = 0.0;
        for (;;) {  // rounds of kRtBlock keys: a one-cell tile may hold more (uniform)
            const uint32_t cc = qi.cc;
            const int nl = active ? qi.cnt : 0;
            const int nfull = nl >> 3, ntail = nl & 7;
            double Fx = 0.0, Fy = 0.0, Fz = 0.0, pe = 0.0, vir = 0.0;
            auto chunk = [&](int c, auto chk_c, int valid) {
                constexpr bool CHK = decltype(chk_c)::value;
                const uint4 raw = raw_a;
                D3 rj[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const uint32_t w = k < 2 ? raw.x : k < 4 ? raw.y : k < 6 ? raw.z : raw.w;
                    uint32_t off = (k & 1) ? w >> 16 : w & 0xffffu;
                    if (CHK && k >= valid) off = 0u;  // padding entries: any record, masked below
                    rj[k] = *reinterpret_cast<const D3*>(sb + off);
                }
                if (!CHK) {
                    raw_a = raw_b;
                    if (8 * (c + 2) < nl) raw_b = ld_stream(l4 + (size_t)(c + 2) * kWave);
                }
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const double dx = rj[k].x - qi.x;
                    const double dy = rj[k].y - qi.y;
                    const double dz = rj[k].z - qi.z;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const bool in = (!CHK || k < valid) && r2 < rc2;
                    double f, e = 0.0;
                    if (fast) {
                        const double xt = __builtin_amdgcn_rcp(r2);
                        const double tt = xt * r2;
                        const double x2 = xt * xt, x3 = x2 * xt, x4 = x2 * x2;
                        const double r8 = x4 * (5.0 - 4.0 * tt), r14 = x4 * x3 * (8.0 - 7.0 * tt);
                        f = in ? 24.0 * r8 - 48.0 * r14 + c2x8 : 0.0;
                        if (ENERGY) e = x3 * x3 * (7.0 - 6.0 * tt) - x3 * (4.0 - 3.0 * tt);
                    } else {
                        const double inv = 1.0 / r2;
                        const double inv3 = inv * inv * inv;
                        f = in ? (24.0 * inv3 - 48.0 * inv3 * inv3) * inv + c2x8 : 0.0;
                        if (ENERGY) e = inv3 * inv3 - inv3;
                    }
                    Fx += f * dx;
                    Fy += f * dy;
                    Fz += f * dz;
                    if (ENERGY) {
                        pe += in ? 2.0 * (e + p.c2 * r2 + p.c0) : 0.0;
                        vir += in ? f * r2 : 0.0;
                    }
                }
            };
            for (int c = 0; c < nfull; ++c) chunk(c, std::false_type{}, U);
            if (ntail) chunk(nfull, std::true_type{}, ntail);
            double ke = 0.0, w2 = 0.0, m2 = 0.0;
            if (active) {
                if (MODE == kForceOnly) {
                    d.fx[key] = Fx;
                    d.fy[key] = Fy;
                    d.fz[key] = Fz;
                    if (ENERGY) ke = 0.5 * p.mass * norm2(v0x, v0y, v0z);
                } else if (MODE == kForceEnd) {
                    const double vx = kick(v0x, p.h, Fx);
                    const double vy = kick(v0y, p.h, Fy);
                    const double vz = kick(v0z, p.h, Fz);
                    d.vx[sp][key] = vx;
                    d.vy[sp][key] = vy;
                    d.vz[sp][key] = vz;
                    d.fx[key] = Fx;
                    d.fy[key] = Fy;
                    d.fz[key] = Fz;
                    if (ENERGY) ke = 0.5 * p.mass * norm2(vx, vy, vz);
                } else {  // kForceMid: close step n, open step n+1, drift
                    const double vx = kick(kick(v0x, p.h, Fx), p.h, Fx);
                    const double vy = kick(kick(v0y, p.h, Fy), p.h, Fy);
                    const double vz = kick(kick(v0z, p.h, Fz), p.h, Fz);
                    st_stream(d.vx[sp] + key, vx);
                    st_stream(d.vy[sp] + key, vy);
                    st_stream(d.vz[sp] + key, vz);
                    const Pos xn = make_pos(drift(qi.x, p.dt, vx), drift(qi.y, p.dt, vy), drift(qi.z, p.dt, vz), cc,
                                            qi.cnt);
                    d.q[sq ^ 1][key] = xn;
                    w2 = norm2(vx, vy, vz);
                    if (d.qb) {
                        const double4 xbq = d.qb[key];
                        m2 = norm2(xn.x - xbq.x, xn.y - xbq.y, xn.z - xbq.z);
                    }
                }
            }
            if (MODE == kForceMid) {
                const double wm = wave_max(w2);
                if (l == 0) stripe_put(d.vmax_s, b, t * 4 + wib, wm);
                if (d.qb) {
                    const double mm = wave_max(m2);
                    if (l == 0) stripe_put(d.disp_s, b, t * 4 + wib, mm);
                }
            }
            if (ENERGY && active) {
                e_ke += ke;
                e_pe += pe;
                e_vir += vir;
            }
            kb += kRtBlock;
            if (kb >= k1) break;
            key = kb + (int)threadIdx.x;
            active = key < k1;
            ks = active ? key : k0;
            qi = d.q[sq][ks];
            v0x = ld_stream(d.vx[sp] + ks);
            v0y = ld_stream(d.vy[sp] + ks);
            v0z = ld_stream(d.vz[sp] + ks);
            l4 = reinterpret_cast<const uint4*>(d.list) + (size_t)(ks >> 6) * p.rows * 8 + (ks & 63);
            raw_a = ld_stream(l4);
            raw_b = p.rows >= 16 ? ld_stream(l4 + kWave) : make_uint4(0u, 0u, 0u, 0u);
        }
        if (ENERGY) {  // the tile's partials, summed in a fixed order
            const double ks2 = wave_sum(e_ke), ps = wave_sum(e_pe), vs = wave_sum(e_vir);
            __syncthreads();
            if (l == 0) {
                red[0][wib] = ks2;
                red[1][wib] = ps;
                red[2][wib] = vs;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double a0 = red[0][0], a1 = red[1][0], a2 = red[2][0];
                for (int w = 1; w < NW; ++w) {
                    a0 += red[0][w];
                    a1 += red[1][w];
                    a2 += red[2][w];
                }
                d.ke_part[t] = a0;
                d.pe_part[t] = a1;
                d.vir_part[t] = a2;
            }
        }
        __syncthreads();  // the next tile's staging reuses the LDS
    }
}

// Half-list steps: F is accumulated by atomics, so the integrator runs as its own
// pass after the force pass.  k_zero_f clears F before the force pass.
__global__ __launch_bounds__(kBlock) void k_zero_f(Dev d, Params p) {
    if (halted(d)) return;
    const int n = p.nwave * kWave;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        d.fx[i] = 0.0;
        d.fy[i] = 0.0;
        d.fz[i] = 0.0;
    }
}

// Closing half kick from stored forces; ENERGY: per-wave kinetic energy partials
// of the kicked velocities (one lane per key, so list waves are slot waves).
template <bool ENERGY>
__global__ __launch_bounds__(kBlock) void k_kick_close(Dev d, Params p) {
    if (halted(d)) return;
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        const int sp = d.st[b].sp;
        double ke = 0.0;
        if (s - g.slot_off < g.npart) {
            const double vx = kick(d.vx[sp][s], p.h, d.fx[s]);
            const double vy = kick(d.vy[sp][s], p.h, d.fy[s]);
            const double vz = kick(d.vz[sp][s], p.h, d.fz[s]);
            d.vx[sp][s] = vx;
            d.vy[sp][s] = vy;
            d.vz[sp][s] = vz;
            if (ENERGY) ke = 0.5 * p.mass * norm2(vx, vy, vz);
        }
        if (ENERGY) {
            const double ks = wave_sum(ke);
            if (l == 0) d.ke_part[w] = ks;
        }
    }
}

// First half kick and drift from stored forces (start of a chunk of steps).
// CLOSE (half-list continuing steps): the closing half kick of the previous step
// first, with the same forces, as the fused full-list pass does.
template <bool CLOSE>
__global__ __launch_bounds__(kBlock) void k_kick_drift(Dev d, Params p) {
    if (halted(d)) return;
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        const int sq = d.st[b].sq, sp = d.st[b].sp;
        double w2 = 0.0, m2 = 0.0;
        if (s - g.slot_off < g.npart) {
            const double vs = d.st[b].vscale;  // thermostat factor; 1 (exact) otherwise
            const double fx = d.fx[s], fy = d.fy[s], fz = d.fz[s];
            const double ux = CLOSE ? kick(d.vx[sp][s], p.h, fx) : d.vx[sp][s];
            const double uy = CLOSE ? kick(d.vy[sp][s], p.h, fy) : d.vy[sp][s];
            const double uz = CLOSE ? kick(d.vz[sp][s], p.h, fz) : d.vz[sp][s];
            const double vx = kick(scale(ux, vs), p.h, fx);
            const double vy = kick(scale(uy, vs), p.h, fy);
            const double vz = kick(scale(uz, vs), p.h, fz);
            d.vx[sp][s] = vx;
            d.vy[sp][s] = vy;
            d.vz[sp][s] = vz;
            const Pos x = d.q[sq][s];
            const Pos xn = make_pos(drift(x.x, p.dt, vx), drift(x.y, p.dt, vy), drift(x.z, p.dt, vz), x.cc, x.cnt);
            d.q[sq ^ 1][s] = xn;
            if (p.precision == MD_PREC_FP32_MIXED) put_u(d.u[sq ^ 1], s, units3(xn, x.cc, g));
            w2 = norm2(vx, vy, vz);
            if (d.qb) {
                const double4 xb = d.qb[s];
                m2 = norm2(xn.x - xb.x, xn.y - xb.y, xn.z - xb.z);
            }
        }
        const double wm = wave_max(w2);
        if (l == 0) stripe_put(d.vmax_s, b, w, wm);
        if (d.qb) {
            const double mm = wave_max(m2);
            if (l == 0) stripe_put(d.disp_s, b, w, mm);
        }
    }
}

// Per-box energies from per-wave partials, in a fixed order (deterministic).
// Per box: KE, PE and pair virial from the per-wave partials in a fixed order;
// optionally the Nose-Hoover half steps around the step boundary (one thread per
// box, the velocity factor left in BoxState::vscale) and a sample of the series.
// Thermostat half step of length h: xi += (h/2) G; factor exp(-xi h) (KE scales by
// its square); eta += xi h; xi += (h/2) G, with G = (2 KE - g T) / Q, g = 3N - 3.
// First level: block (j, b) sums segment j (kRedSeg partials) of box b in a fixed
// order, so the two-level total is the same on every run.
__device__ __forceinline__ void block_sum3(double& k, double& e, double& v) {
    __shared__ double ks[kBlock], ps[kBlock], vs[kBlock];
    ks[threadIdx.x] = k;
    ps[threadIdx.x] = e;
    vs[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            ks[threadIdx.x] += ks[threadIdx.x + o];
            ps[threadIdx.x] += ps[threadIdx.x + o];
            vs[threadIdx.x] += vs[threadIdx.x + o];
        }
        __syncthreads();
    }
    k = ks[0];
    e = ps[0];
    v = vs[0];
    __syncthreads();
}

// Partials of box b: per list wavefront (K = 64 / tpk keys each), or per row tile
// (tl) when the row-tile force kernel wrote them.
__device__ __forceinline__ void part_range(const Dev& d, const Params& p, const BoxGeom& g, int b, int tl, int& w0,
                                           int& w1) {
    if (tl) {
        w0 = d.box_t0[b];
        w1 = d.box_t0[b + 1];
    } else {
        const int K = kWave / p.tpk;
        w0 = g.slot_off / K;
        w1 = (g.slot_off + g.nslot) / K;
    }
}

__global__ __launch_bounds__(kBlock) void k_energy_segments(Dev d, Params p, int tl) {
    if (halted(d)) return;
    const int b = blockIdx.y, j = blockIdx.x;
    const BoxGeom& g = d.geom[b];
    int w0, w1;
    part_range(d, p, g, b, tl, w0, w1);
    const int a0 = w0 + j * kRedSeg, a1 = min(a0 + kRedSeg, w1);
    if (a0 >= w1) return;  // uniform over the block
    double k = 0.0, e = 0.0, v = 0.0;
    for (int w = a0 + threadIdx.x; w < a1; w += kBlock) {
        k += d.ke_part[w];
        e += d.pe_part[w];
        v += d.vir_part[w];
    }
    block_sum3(k, e, v);
    if (threadIdx.x == 0) {
        double* r = d.red + ((size_t)b * p.redcap + j) * 3;
        r[0] = k;
        r[1] = e;
        r[2] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_energy_reduce(Dev d, Params p, int record, int thermo, int tl) {
    if (halted(d)) return;
    for (int b = blockIdx.x; b < p.nbox; b += gridDim.x) {
        const BoxGeom& g = d.geom[b];
        int w0, w1;
        part_range(d, p, g, b, tl, w0, w1);
        const int nseg = (w1 - w0 + kRedSeg - 1) / kRedSeg;
        double k = 0.0, e = 0.0, v = 0.0;
        for (int j = threadIdx.x; j < nseg; j += kBlock) {
            const double* r = d.red + ((size_t)b * p.redcap + j) * 3;
            k += r[0];
            e += r[1];
            v += r[2];
        }
        block_sum3(k, e, v);
        if (threadIdx.x == 0) {
            BoxState& st = d.st[b];
            double ke = k, ke_s = k, th = 0.0;  // ke_s, th: values at the sample time
            if (thermo && st.thQ > 0.0) {
                const double gT = (3.0 * g.npart - 3.0) * st.thT, Q = st.thQ, h = 0.5 * p.dt;
                double xi = st.xi, eta = st.eta, f = 1.0;
                for (int half = 0; half < 2; ++half) {  // 0: ends this step, 1: starts the next
                    if (!(thermo & (1 << half))) continue;
                    xi = xi + 0.5 * h * ((2.0 * ke - gT) / Q);
                    const double sc = exp(-xi * h);
                    f = f * sc;
                    ke = ke * (sc * sc);
                    eta = eta + xi * h;
                    xi = xi + 0.5 * h * ((2.0 * ke - gT) / Q);
                    if (half == 0) {
                        ke_s = ke;
                        th = 0.5 * Q * xi * xi + gT * eta;
                    }
                }
                st.xi = xi;
                st.eta = eta;
                st.vscale = f;
            }
            st.ke = ke_s;
            st.pe = e;
            st.vir = 0.5 * v;  // every pair appears in both keys' lists
            if (record && st.nseries < kMaxSeries) {
                const size_t at = (size_t)st.nseries * p.nbox + b;
                d.series_ke[at] = ke_s;
                d.series_pe[at] = e;
                d.series_vir[at] = 0.5 * v;
                d.series_th[at] = th;
                st.nseries += 1;
            }
        }
        __syncthreads();
    }
}

// KE partials of the current velocities, in the per-list-wave layout the
// reduction reads (a slot wave's sum in its first list wave, zeros in the others).
__global__ __launch_bounds__(kBlock) void k_ke_partial(Dev d, Params p) {
    if (halted(d)) return;
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l, sp = d.st[b].sp;
        const double k = s - g.slot_off < g.npart ? 0.5 * p.mass * norm2(d.vx[sp][s], d.vy[sp][s], d.vz[sp][s])
                                                  : 0.0;
        const double ks = wave_sum(k);
        if (l < p.tpk) {
            d.ke_part[w * p.tpk + l] = l == 0 ? ks : 0.0;
            d.pe_part[w * p.tpk + l] = 0.0;
            d.vir_part[w * p.tpk + l] = 0.0;
        }
    }
}

// Apply the pending thermostat factor to the velocities (end of a run of steps).
__global__ __launch_bounds__(kBlock) void k_vscale(Dev d, Params p) {
    if (halted(d)) return;
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l, sp = d.st[b].sp;
        if (s - g.slot_off >= g.npart) continue;
        const double f = d.st[b].vscale;
        d.vx[sp][s] = scale(d.vx[sp][s], f);
        d.vy[sp][s] = scale(d.vy[sp][s], f);
        d.vz[sp][s] = scale(d.vz[sp][s], f);
    }
}

// Debug verifier: pairs within rc (minimum image, current positions) that the
// key's list lacks.  O(n^2) per box.
__global__ __launch_bounds__(kBlock) void k_verify(Dev d, Params p) {
    if (halted(d)) return;
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        if (s - g.slot_off >= g.npart) continue;
        const Pos* q = d.q[d.st[b].sq];
        const Pos qi = q[s];
        const int n = d.cnt[s];
        int ps0[27], plen[27];
        if (p.tile) tile_pieces_of(d, g, qi.cc, ps0, plen);
        unsigned long long missed = 0;
        for (int j = g.slot_off; j < g.slot_off + g.npart; ++j) {
            if (j == s) continue;
            const Pos qj = q[j];
            double t[3] = {qj.x - qi.x, qj.y - qi.y, qj.z - qi.z};
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double dd = t[a] - g.L[a] * rint(t[a] / g.L[a]);
                r2 += dd * dd;
            }
            if (r2 < p.rc2) {
                bool found = false;
                for (int e = 0; e < n && !found; ++e) {
                    const uint32_t en = d.list[list_addr(s, e, p.tpk, p.rows)];
                    found = (p.tile ? tile_slot(ps0, plen, en, p.recb) : entry_slot(d, qi.cc, en, g)) == j;
                }
                if (!found) ++missed;
            }
        }
        if (missed) atomicAdd(&d.st[b].missed, missed);
    }
}

__global__ __launch_bounds__(kBlock) void k_scale(Dev d, Params p, const double* __restrict__ alpha_q,
                                                  const double* __restrict__ scale_v) {
    const int l = lane_id();
    for (int w = blockIdx.x * 4 + wave_in_block(); w < p.nwave; w += gridDim.x * 4) {
        const int b = ld_const(d.wave_box + w);
        const BoxGeom& g = d.geom[b];
        const int s = w * kWave + l;
        if (s - g.slot_off >= g.npart) continue;
        const int sq = d.st[b].sq, sp = d.st[b].sp;
        if (alpha_q) {
            const double a = alpha_q[b];
            Pos x = d.q[sq][s];
            x.x *= a;
            x.y *= a;
            x.z *= a;
            d.q[sq][s] = x;
        }
        if (scale_v) {
            const double c = scale_v[b];
            d.vx[sp][s] *= c;
            d.vy[sp][s] *= c;
            d.vz[sp][s] *= c;
        }
    }
}

// A larger list buffer: every slot's entries moved from the old layout (old_rows
// chunks of 8 per list lane) to the current one (p.rows), so the boxes that do not
// rebuild at the step an overflow stopped keep their lists.  One thread per slot;
// entry e < min(cnt, old capacity) exists in both layouts.
__global__ __launch_bounds__(kBlock) void k_list_relayout(Dev d, Params p, const uint16_t* __restrict__ old,
                                                          int old_rows) {
    const int nslot = p.nwave * kWave;
    const int old_cap = old_rows * p.tpk;
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < nslot; s += gridDim.x * kBlock) {
        const int n = min(max(d.cnt[s], 0), old_cap);
        for (int e = 0; e < n; ++e) d.list[list_addr(s, e, p.tpk, p.rows)] = old[list_addr(s, e, p.tpk, old_rows)];
    }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------- launchers

static inline int grid_for_waves(int nwave, int cap = 4096) {
    int g = (nwave + 3) / 4;
    return g < 1 ? 1 : (g > cap ? cap : g);
}

void launch_set_state(const Dev& d, const Params& p, const double* pos, const double* vel, int32_t nwave,
                      hipStream_t s) {
    k_set_state<<<grid_for_waves(nwave), kBlock, 0, s>>>(d, p, pos, vel);
}
void launch_get_state(const Dev& d, const Params& p, double* pos, double* vel, int32_t nwave, hipStream_t s) {
    k_get_state<<<grid_for_waves(nwave), kBlock, 0, s>>>(d, p, pos, vel);
}
void launch_get_forces(const Dev& d, const Params& p, double* f, int32_t nwave, hipStream_t s) {
    k_get_forces<<<grid_for_waves(nwave), kBlock, 0, s>>>(d, p, f);
}
void launch_get_cells(const Dev& d, const Params& p, int32_t* c, int32_t nwave, hipStream_t s) {
    k_get_cells<<<grid_for_waves(nwave), kBlock, 0, s>>>(d, p, c);
}
void launch_list_counts(const Dev& d, const Params& p, int64_t* c, int32_t nwave, hipStream_t s) {
    k_list_counts<<<grid_for_waves(nwave), kBlock, 0, s>>>(d, p, c);
}
void launch_list_export(const Dev& d, const Params& p, const int64_t* kp, int32_t* partners, int32_t nwave,
                        hipStream_t s) {
    k_list_export<<<grid_for_waves(nwave), kBlock, 0, s>>>(d, p, kp, partners);
}
void launch_mark_rebuild(const Dev& d, const Params& p, hipStream_t s) {
    k_mark_rebuild<<<1, kBlock, 0, s>>>(d, p);
}

// List-build grid: each wavefront takes about 8 cells (a block 32), between 8192 and 65536
// blocks.  Fewer, longer-lived wavefronts ran slower at 32M particles (rebuild chain 8.37 ms
// with 8192 blocks, 9.42 ms with one resident round of 1792), and so did one cell per
// wavefront (8.69 ms); 32768-65536 blocks gave 7.88-7.92 ms.  The lower bound keeps the
// grid of smaller boxes as it was (unchanged at 1M particles, 4% faster build at 4M).
static inline int list_grid(const Params& p) {
    const int g = p.ntile * kTile / 32;
    return g < 8192 ? grid_for_waves(p.ntile * kTile, 8192) : (g > 65536 ? 65536 : g);
}
template <int TPK>
static void launch_list_t(const Dev& d, const Params& p, hipStream_t s) {
    if (TPK == 1 && p.half)
        k_list<1, true, false><<<list_grid(p), kBlock, 0, s>>>(d, p);
    else if (TPK == 1 && p.tile)
        k_list<1, false, true><<<list_grid(p), kBlock, 0, s>>>(d, p);
    else
        k_list<TPK, false, false><<<list_grid(p), kBlock, 0, s>>>(d, p);
}

void launch_row_tiles(const Dev& d, const Params& p, hipStream_t s) {
    const int gr = grid_for_waves(p.nrows);
    k_row_tiles<<<gr, kBlock, 0, s>>>(d, p);
    k_row_scan<<<1, kBlock, 0, s>>>(d, p);
    k_row_write<<<gr, kBlock, 0, s>>>(d, p);
    k_row_delta<<<4096, kBlock, 0, s>>>(d, p);
}

void launch_rebuild_chain(const Dev& d, const Params& p, bool with_list, hipStream_t s) {
    const int gw = grid_for_waves(p.nwave);
    const int gt = p.ntile < 4096 ? p.ntile : 4096;
    k_cell_clear<<<gt, kBlock, 0, s>>>(d, p);
    k_bin<<<gw, kBlock, 0, s>>>(d, p);
    k_scan_tile<<<gt, kBlock, 0, s>>>(d, p);
    k_scan_box<<<p.nbox < 1024 ? p.nbox : 1024, kBlock, 0, s>>>(d, p);
    k_scan_add<<<gt, kBlock, 0, s>>>(d, p);
    if (p.tile) launch_row_tiles(d, p, s);
    k_scatter<<<gw, kBlock, 0, s>>>(d, p);
    k_rank_permute<<<gw, kBlock, 0, s>>>(d, p);
    if (with_list) {
        switch (p.tpk) {
            case 1: launch_list_t<1>(d, p, s); break;
            case 2: launch_list_t<2>(d, p, s); break;
            case 4: launch_list_t<4>(d, p, s); break;
            default: launch_list_t<8>(d, p, s); break;
        }
    }
    k_post_build<<<p.nbox < 1024 ? p.nbox : 1024, kBlock, 0, s>>>(d, p, with_list ? 1 : 0);
}

template <int PREC, int TPK>
static void launch_force_pt(const Dev& d, const Params& p, int mode, bool energy, hipStream_t s) {
    const int nb = (p.nwave * TPK + 3) / 4;
    if (mode == kForceOnly) {
        if (energy)
            k_force<PREC, kForceOnly, TPK, true><<<nb, kBlock, 0, s>>>(d, p);
        else
            k_force<PREC, kForceOnly, TPK, false><<<nb, kBlock, 0, s>>>(d, p);
    } else if (mode == kForceEnd) {
        if (energy)
            k_force<PREC, kForceEnd, TPK, true><<<nb, kBlock, 0, s>>>(d, p);
        else
            k_force<PREC, kForceEnd, TPK, false><<<nb, kBlock, 0, s>>>(d, p);
    } else {
        k_force<PREC, kForceMid, TPK, false><<<nb, kBlock, 0, s>>>(d, p);
    }
}

template <int PREC>
static void launch_force_p(const Dev& d, const Params& p, int mode, bool energy, hipStream_t s) {
    switch (p.tpk) {
        case 1: launch_force_pt<PREC, 1>(d, p, mode, energy, s); break;
        case 2: launch_force_pt<PREC, 2>(d, p, mode, energy, s); break;
        case 4: launch_force_pt<PREC, 4>(d, p, mode, energy, s); break;
        default: launch_force_pt<PREC, 8>(d, p, mode, energy, s); break;
    }
}

// Half list: clear F, accumulate it with the reactions, then integrate from it.
template <int PREC>
static void launch_force_half(const Dev& d, const Params& p, int mode, bool energy, hipStream_t s) {
    const int nb = (p.nwave + 3) / 4;
    k_zero_f<<<grid_for_waves(p.nwave), kBlock, 0, s>>>(d, p);
    if (energy)
        k_force<PREC, kForceOnly, 1, true, true><<<nb, kBlock, 0, s>>>(d, p);
    else
        k_force<PREC, kForceOnly, 1, false, true><<<nb, kBlock, 0, s>>>(d, p);
    if (mode == kForceEnd) {
        if (energy)
            k_kick_close<true><<<nb, kBlock, 0, s>>>(d, p);
        else
            k_kick_close<false><<<nb, kBlock, 0, s>>>(d, p);
    } else if (mode == kForceMid) {
        k_kick_drift<true><<<nb, kBlock, 0, s>>>(d, p);
    }
}

template <bool CLAMP>
static void launch_force_rowtile_c(const Dev& d, const Params& p, int mode, bool energy, hipStream_t s) {
    const size_t lds = (size_t)p.scap * sizeof(U3);
    if (mode == kForceOnly) {
        if (energy)
            k_force_t<kForceOnly, true, CLAMP><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
        else
            k_force_t<kForceOnly, false, CLAMP><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
    } else if (mode == kForceEnd) {
        if (energy)
            k_force_t<kForceEnd, true, CLAMP><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
        else
            k_force_t<kForceEnd, false, CLAMP><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
    } else {
        k_force_t<kForceMid, false, CLAMP><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
    }
}

// Resident blocks per compute unit of the mid-step row-tile kernel with its LDS: the
// row-tile kernels launch that many blocks per CU, and each loops over the tiles.
int rowtile_blocks_per_cu(const Params& p) {
    int nb = 0;
    hipError_t e;
    if (p.precision == MD_PREC_FP64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force_t64<kForceMid, false>, kRtBlock,
                                                         (size_t)p.scap * sizeof(D3));
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force_t<kForceMid, false, true>, kRtBlock,
                                                         (size_t)p.scap * sizeof(U3));
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

static void launch_force_rowtile64(const Dev& d, const Params& p, int mode, bool energy, hipStream_t s) {
    const size_t lds = (size_t)p.scap * sizeof(D3);
    if (mode == kForceOnly) {
        if (energy)
            k_force_t64<kForceOnly, true><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
        else
            k_force_t64<kForceOnly, false><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
    } else if (mode == kForceEnd) {
        if (energy)
            k_force_t64<kForceEnd, true><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
        else
            k_force_t64<kForceEnd, false><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
    } else {
        k_force_t64<kForceMid, false><<<p.tgrid, kRtBlock, lds, s>>>(d, p);
    }
}

static void launch_force_rowtile(const Dev& d, const Params& p, int mode, bool energy, hipStream_t s) {
    if (p.precision == MD_PREC_FP64)
        launch_force_rowtile64(d, p, mode, energy, s);
    else if (p.clamp)
        launch_force_rowtile_c<true>(d, p, mode, energy, s);
    else
        launch_force_rowtile_c<false>(d, p, mode, energy, s);
}

void launch_force(const Dev& d, const Params& p, int mode, bool energy, hipStream_t s) {
    if (p.tile) return launch_force_rowtile(d, p, mode, energy, s);
    if (p.half) {
        if (p.precision == MD_PREC_FP64)
            launch_force_half<MD_PREC_FP64>(d, p, mode, energy, s);
        else
            launch_force_half<MD_PREC_FP32_MIXED>(d, p, mode, energy, s);
        return;
    }
    if (p.precision == MD_PREC_FP64)
        launch_force_p<MD_PREC_FP64>(d, p, mode, energy, s);
    else
        launch_force_p<MD_PREC_FP32_MIXED>(d, p, mode, energy, s);
}

void launch_kick_drift(const Dev& d, const Params& p, hipStream_t s) {
    k_kick_drift<false><<<(p.nwave + 3) / 4, kBlock, 0, s>>>(d, p);
}
void launch_dutc(const Dev& d, const Params& p, hipStream_t s) {
    k_dutc<<<p.nbox < 1024 ? p.nbox : 1024, kBlock, 0, s>>>(d, p);
}
void launch_energy_reduce(const Dev& d, const Params& p, bool record, int thermo, bool tl, hipStream_t s) {
    const int nparts = tl ? p.maxcell : p.maxslot / kWave * p.tpk;  // a box has at most one row tile per cell
    const int nseg = (nparts + kRedSeg - 1) / kRedSeg;
    k_energy_segments<<<dim3(nseg, p.nbox), kBlock, 0, s>>>(d, p, tl ? 1 : 0);
    k_energy_reduce<<<p.nbox < 1024 ? p.nbox : 1024, kBlock, 0, s>>>(d, p, record ? 1 : 0, thermo, tl ? 1 : 0);
}
void launch_ke_partial(const Dev& d, const Params& p, hipStream_t s) {
    k_ke_partial<<<grid_for_waves(p.nwave), kBlock, 0, s>>>(d, p);
}
void launch_vscale(const Dev& d, const Params& p, hipStream_t s) {
    k_vscale<<<grid_for_waves(p.nwave), kBlock, 0, s>>>(d, p);
}
void launch_verify(const Dev& d, const Params& p, hipStream_t s) {
    k_verify<<<grid_for_waves(p.nwave), kBlock, 0, s>>>(d, p);
}
void launch_scale(const Dev& d, const Params& p, const double* alpha_q, const double* scale_v, hipStream_t s) {
    k_scale<<<grid_for_waves(p.nwave), kBlock, 0, s>>>(d, p, alpha_q, scale_v);
}
void launch_list_relayout(const Dev& d, const Params& p, const uint16_t* old, int32_t old_rows, hipStream_t s) {
    k_list_relayout<<<grid_for_waves(p.nwave), kBlock, 0, s>>>(d, p, old, old_rows);
}
void launch_fill_i32(int32_t* ptr, int32_t v, int64_t n, hipStream_t s) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    k_fill_i32<<<(int)g, kBlock, 0, s>>>(ptr, v, n);
}

}  // namespace mdg
