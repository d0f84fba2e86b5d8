// md_bubbles.hip -- bubble identification on the GPU (Sec. IV.B).
//
// The analysis of the cavitation runs: particles are counted per subcell of
// edge >= 3 into one byte each, a subcell whose count is below the gas density
// times its volume is gas, and gas subcells that share a face belong to one
// bubble (site percolation on the periodic simple cubic lattice).  The paper
// gathers the byte field to one process and clusters it serially; here the
// field never leaves the GPU:
//
//   k_sub_count  one thread per particle: wrap, bin, atomic count per subcell
//   k_sub_flags  byte count (saturating), gas flag -> parent[i] = i or -1
//   k_sub_hook   one thread per gas subcell: union with its +x, +y, +z
//                neighbours (periodic) in a lock-free union-find whose links
//                always point to a smaller index, so a bubble's final root is
//                its smallest subcell index
//   k_sub_label  label = root (path halving on the way), sizes by atomics
//   k_sub_roots  compacts (root, size) pairs; the host sorts them by root
//
// Union-find on the GPU after the published lock-free scheme of linking a root
// to a smaller root with compare-and-swap and compressing paths with plain
// ancestor stores (connected components as in ECL-CC, Jaiganesh and Burtscher,
// HPDC 2018).  Every parent pointer only ever moves to an ancestor, so every
// loop terminates: finds follow strictly decreasing indices, and each failed
// compare-and-swap means another thread's link succeeded.
#include "md.h"
#include "md_internal.h"

namespace mdg {

__device__ __forceinline__ int32_t ld_rlx(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rlx(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x; every node passed points to its grandparent afterwards.
__device__ __forceinline__ int32_t find_root(int32_t* par, int32_t x) {
    int32_t p = ld_rlx(par + x);
    while (p != x) {
        const int32_t gp = ld_rlx(par + p);
        if (gp != p) st_rlx(par + x, gp);
        x = p;
        p = gp;
    }
    return x;
}

__device__ __forceinline__ void unite(int32_t* par, int32_t a, int32_t b) {
    int32_t ra = find_root(par, a), rb = find_root(par, b);
    while (ra != rb) {
        if (ra < rb) {
            const int32_t t = ra;
            ra = rb;
            rb = t;
        }
        const int32_t old = atomicCAS(par + ra, ra, rb);  // hang the larger root below the smaller
        if (old == ra) return;
        ra = find_root(par, old);
        rb = find_root(par, rb);
    }
}

__global__ __launch_bounds__(kBlock) void k_sub_count(Dev d, int32_t b, SubGrid sg, uint32_t* __restrict__ cnt,
                                                      int32_t* __restrict__ flag) {
    const BoxGeom& g = d.geom[b];
    const int sq = d.st[b].sq;
    const Pos* __restrict__ q = d.q[sq] + g.slot_off;
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < g.npart; k += gridDim.x * kBlock) {
        const Pos x = q[k];
        double c0 = x.x, c1 = x.y, c2 = x.z;
        bool bad = false;
        const int cx = bin_axis(c0, sg.L[0], sg.inv[0], sg.n[0], bad);
        const int cy = bin_axis(c1, sg.L[1], sg.inv[1], sg.n[1], bad);
        const int cz = bin_axis(c2, sg.L[2], sg.inv[2], sg.n[2], bad);
        if (bad) {
            atomicOr(flag, 1);
            continue;
        }
        atomicAdd(cnt + ((cz * sg.n[1] + cy) * sg.n[0] + cx), 1u);
    }
}

__global__ __launch_bounds__(kBlock) void k_sub_flags(SubGrid sg, const uint32_t* __restrict__ cnt,
                                                      uint8_t* __restrict__ bytes, int32_t* __restrict__ par,
                                                      int32_t* __restrict__ size) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < sg.nsub; i += gridDim.x * kBlock) {
        const uint32_t c = cnt[i] > 255u ? 255u : cnt[i];
        if (bytes) bytes[i] = (uint8_t)c;
        par[i] = (double)c < sg.thr ? i : -1;
        size[i] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_sub_hook(SubGrid sg, int32_t* __restrict__ par) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < sg.nsub; i += gridDim.x * kBlock) {
        if (ld_rlx(par + i) < 0) continue;  // liquid; a gas subcell's pointer is never negative
        const int x = i % sg.n[0];
        const int y = (i / sg.n[0]) % sg.n[1];
        const int z = i / (sg.n[0] * sg.n[1]);
        const int nb[3] = {(z * sg.n[1] + y) * sg.n[0] + (x + 1 == sg.n[0] ? 0 : x + 1),
                           (z * sg.n[1] + (y + 1 == sg.n[1] ? 0 : y + 1)) * sg.n[0] + x,
                           ((z + 1 == sg.n[2] ? 0 : z + 1) * sg.n[1] + y) * sg.n[0] + x};
        for (int a = 0; a < 3; ++a) {
            const int j = nb[a];
            if (j != i && ld_rlx(par + j) >= 0) unite(par, i, j);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_sub_label(SubGrid sg, int32_t* __restrict__ par,
                                                      int32_t* __restrict__ lab, int32_t* __restrict__ size) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < sg.nsub; i += gridDim.x * kBlock) {
        if (ld_rlx(par + i) < 0) {
            lab[i] = -1;
            continue;
        }
        const int32_t r = find_root(par, i);
        lab[i] = r;
        atomicAdd(size + r, 1);
    }
}

__global__ __launch_bounds__(kBlock) void k_sub_roots(SubGrid sg, const int32_t* __restrict__ lab,
                                                      const int32_t* __restrict__ size, int2* __restrict__ out,
                                                      int32_t* __restrict__ count) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < sg.nsub; i += gridDim.x * kBlock) {
        if (lab[i] != i) continue;
        const int32_t k = atomicAdd(count, 1);  // < nsub: at most one entry per subcell
        out[k] = make_int2(i, size[i]);
    }
}

static int grid_for(int64_t n) {
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
}

void launch_bubbles(const Dev& d, int32_t b, int32_t npart, const SubGrid& sg, const BubbleWork& w, uint8_t* bytes,
                    hipStream_t s) {
    k_sub_count<<<grid_for(npart), kBlock, 0, s>>>(d, b, sg, w.cnt, w.flag);
    k_sub_flags<<<grid_for(sg.nsub), kBlock, 0, s>>>(sg, w.cnt, bytes, w.par, w.size);
    k_sub_hook<<<grid_for(sg.nsub), kBlock, 0, s>>>(sg, w.par);
    k_sub_label<<<grid_for(sg.nsub), kBlock, 0, s>>>(sg, w.par, w.lab, w.size);
    k_sub_roots<<<grid_for(sg.nsub), kBlock, 0, s>>>(sg, w.lab, w.size, w.roots, w.flag + 1);
}

}  // namespace mdg
