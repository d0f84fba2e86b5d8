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
// md_bubbles_noalloc runs the same count / flag / hook / label kernels on a
// fixed device array instead of allocated buffers and replaces the last step by
// an ordered compaction (root counts per segment, one-block scan, write-out in
// subcell order), so the bubbles arrive sorted without a host-side buffer.
//
// Union-find on the GPU after the published lock-free scheme of linking a root
// to a smaller root with compare-and-swap and compressing paths with plain
// ancestor stores (connected components as in ECL-CC, Jaiganesh and Burtscher,
// HPDC 2018).  Every parent pointer only ever moves to an ancestor, so every
// loop terminates: finds follow strictly decreasing indices, and each failed
// compare-and-swap means another thread's link succeeded.
#include <mutex>

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

// ---------------------------------------------------------------- fixed scratch
//
// The allocation-free variant (md_bubbles_noalloc) keeps every work buffer in one
// file-scope device array.  In host code `scratch` is only a host-side stand-in:
// its device address is taken once per device with hipGetSymbolAddress
// (bubbles_scratch_init) and only that address is ever handed to kernels.
// Layout (kNaMaxSub subcells): cnt u32, par i32, lab i32, size i32, root i64,
// rsize i64 per subcell, then the per-segment root counts and offsets of the
// ordered compaction, then the status words.
constexpr size_t kNaCnt = 0;
constexpr size_t kNaPar = kNaCnt + 4 * (size_t)kNaMaxSub;
constexpr size_t kNaLab = kNaPar + 4 * (size_t)kNaMaxSub;
constexpr size_t kNaSize = kNaLab + 4 * (size_t)kNaMaxSub;
constexpr size_t kNaRoot = kNaSize + 4 * (size_t)kNaMaxSub;
constexpr size_t kNaRsize = kNaRoot + 8 * (size_t)kNaMaxSub;
constexpr size_t kNaSegCnt = kNaRsize + 8 * (size_t)kNaMaxSub;
constexpr size_t kNaSegOff = kNaSegCnt + 4 * (size_t)kNaSegs;
constexpr size_t kNaMisc = kNaSegOff + 4 * (size_t)kNaSegs;
constexpr size_t kNaBytes = kNaMisc + sizeof(NaMisc);
static_assert(kNaMaxSub % kNaSeg == 0, "whole segments");
static_assert(kNaSegs <= kBlock * 4, "one block scans the segment counts");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_na_mu;
unsigned char* g_na_ptr[kMaxDevices] = {};
}  // namespace

hipError_t bubbles_scratch_init(int device) {
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_na_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_na_ptr[device] = static_cast<unsigned char*>(p);
    return hipSuccess;
}

unsigned char* bubbles_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_na_mu);
    return device >= 0 && device < kMaxDevices ? g_na_ptr[device] : nullptr;
}

BubbleWork bubbles_scratch_work(unsigned char* base) {
    BubbleWork w{};
    w.cnt = reinterpret_cast<uint32_t*>(base + kNaCnt);
    w.par = reinterpret_cast<int32_t*>(base + kNaPar);
    w.lab = reinterpret_cast<int32_t*>(base + kNaLab);
    w.size = reinterpret_cast<int32_t*>(base + kNaSize);
    w.roots = nullptr;  // the ordered compaction writes root / rsize instead
    w.flag = reinterpret_cast<int32_t*>(base + kNaMisc);  // NaMisc::bad
    return w;
}

// Clears the per-subcell counters and the status words (a fill kernel, not a
// memset, so the sequence may be captured in a graph).
__global__ __launch_bounds__(kBlock) void k_na_clear(uint32_t* __restrict__ cnt, int32_t nsub, NaMisc* misc) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nsub; i += gridDim.x * kBlock) cnt[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) *misc = NaMisc{};
}

// Roots (lab[i] == i) per segment of kNaSeg subcells; gas subcells and the largest
// bubble by atomics (order-independent).
__global__ __launch_bounds__(kBlock) void k_na_segcount(SubGrid sg, const int32_t* __restrict__ lab,
                                                        const int32_t* __restrict__ size,
                                                        int32_t* __restrict__ segcnt, NaMisc* misc) {
    __shared__ int red[kBlock];
    const int s = blockIdx.x;
    const int i0 = s * kNaSeg, i1 = min(i0 + kNaSeg, sg.nsub);
    int nr = 0, ng = 0, big = 0;
    for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
        const int32_t r = lab[i];
        ng += r >= 0 ? 1 : 0;
        if (r == i) {
            nr += 1;
            big = max(big, size[i]);
        }
    }
    red[threadIdx.x] = nr;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) segcnt[s] = red[0];
    if (ng) atomicAdd(&misc->ngas, (unsigned long long)ng);
    if (big) atomicMax(&misc->largest, big);
}

// One block: exclusive scan of the segment counts; the total is the bubble count.
__global__ __launch_bounds__(kBlock) void k_na_segscan(int32_t nseg, const int32_t* __restrict__ segcnt,
                                                       int32_t* __restrict__ segoff, NaMisc* misc) {
    __shared__ int part[kBlock];
    constexpr int kPer = 4;  // segments per thread (nseg <= kBlock * kPer)
    int v[kPer], tot = 0;
    for (int k = 0; k < kPer; ++k) {
        const int j = threadIdx.x * kPer + k;
        v[k] = j < nseg ? segcnt[j] : 0;
        tot += v[k];
    }
    part[threadIdx.x] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < kBlock; ++t) {
            const int x = part[t];
            part[t] = run;
            run += x;
        }
        misc->nroots = run;
    }
    __syncthreads();
    int run = part[threadIdx.x];
    for (int k = 0; k < kPer; ++k) {
        const int j = threadIdx.x * kPer + k;
        if (j < nseg) segoff[j] = run;
        run += v[k];
    }
}

// Roots of each segment in ascending subcell order at the segment's offset.
__global__ __launch_bounds__(kBlock) void k_na_segwrite(SubGrid sg, const int32_t* __restrict__ lab,
                                                        const int32_t* __restrict__ size,
                                                        const int32_t* __restrict__ segoff,
                                                        int64_t* __restrict__ root, int64_t* __restrict__ rsize) {
    __shared__ int part[kBlock];
    constexpr int kPer = kNaSeg / kBlock;  // consecutive subcells per thread
    const int s = blockIdx.x;
    const int i0 = s * kNaSeg + threadIdx.x * kPer;
    int n = 0;
    for (int k = 0; k < kPer; ++k) {
        const int i = i0 + k;
        n += (i < sg.nsub && lab[i] == i) ? 1 : 0;
    }
    part[threadIdx.x] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < kBlock; ++t) {
            const int x = part[t];
            part[t] = run;
            run += x;
        }
    }
    __syncthreads();
    int at = segoff[s] + part[threadIdx.x];
    for (int k = 0; k < kPer; ++k) {
        const int i = i0 + k;
        if (i < sg.nsub && lab[i] == i) {
            root[at] = i;
            rsize[at] = size[i];
            ++at;
        }
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

void launch_bubbles_scratch(const Dev& d, int32_t b, int32_t npart, const SubGrid& sg, unsigned char* base,
                            uint8_t* bytes, hipStream_t s) {
    const BubbleWork w = bubbles_scratch_work(base);
    NaMisc* misc = reinterpret_cast<NaMisc*>(base + kNaMisc);
    int32_t* segcnt = reinterpret_cast<int32_t*>(base + kNaSegCnt);
    int32_t* segoff = reinterpret_cast<int32_t*>(base + kNaSegOff);
    const int nseg = (sg.nsub + kNaSeg - 1) / kNaSeg;
    k_na_clear<<<grid_for(sg.nsub), kBlock, 0, s>>>(w.cnt, sg.nsub, misc);
    k_sub_count<<<grid_for(npart), kBlock, 0, s>>>(d, b, sg, w.cnt, &misc->bad);
    k_sub_flags<<<grid_for(sg.nsub), kBlock, 0, s>>>(sg, w.cnt, bytes, w.par, w.size);
    k_sub_hook<<<grid_for(sg.nsub), kBlock, 0, s>>>(sg, w.par);
    k_sub_label<<<grid_for(sg.nsub), kBlock, 0, s>>>(sg, w.par, w.lab, w.size);
    k_na_segcount<<<nseg, kBlock, 0, s>>>(sg, w.lab, w.size, segcnt, misc);
    k_na_segscan<<<1, kBlock, 0, s>>>(nseg, segcnt, segoff, misc);
    k_na_segwrite<<<nseg, kBlock, 0, s>>>(sg, w.lab, w.size, segoff, reinterpret_cast<int64_t*>(base + kNaRoot),
                                          reinterpret_cast<int64_t*>(base + kNaRsize));
}

void bubbles_scratch_results(unsigned char* base, int64_t** root, int64_t** rsize, int32_t** lab, NaMisc** misc) {
    *root = reinterpret_cast<int64_t*>(base + kNaRoot);
    *rsize = reinterpret_cast<int64_t*>(base + kNaRsize);
    *lab = reinterpret_cast<int32_t*>(base + kNaLab);
    *misc = reinterpret_cast<NaMisc*>(base + kNaMisc);
}

}  // namespace mdg
