// md_internal.h -- layouts shared by the host API (md_api.hip) and the gfx950
// kernels (md_kernels.hip).  Not part of the public ABI.
//
// Data layout in HBM (all boxes of a context share each array):
//   slots     particles live in "slots" sorted by cell; box b owns slots
//             [slot_off, slot_off + nslot), nslot = npart rounded up to 64, so a
//             64-lane wavefront never spans two boxes.  Padding slots are idle.
//   q[2]      Pos records (x, y, z in FP64, the packed cell coordinates of the last
//             build, the list length), 32 bytes, ping-pong: the force kernel gathers
//             partners from q[sq] and writes drifted positions to q[1-sq].
//   u[2]      positions in fixed point, 3 int32 per slot (12 bytes, no padding;
//             FP32-mixed path), ping-pong with q: per axis
//             U = c * uoff + rint((x - (c + 1/2) cs) * ucs) modulo 2^32, c = the
//             particle's cell at the last build, uoff = rint(cs * ucs) one cell side
//             in units, ucs a power of two (units per length, the same on every
//             axis).  A pair's separation U_j - U_i - r * n * uoff (r = periodic
//             image) is exact in int32; it is converted to FP32 once, and lengths
//             stay in units until the per-particle force is scaled back.
//   v*[2]     float64 velocity components (SoA), ping-pong only across a re-sort.
//   id[2]     caller index of the particle in each slot.
//   list      wave-blocked ELL pair list of 16-bit entries.  A list wave holds
//             K = 64 / tpk keys and rows * 64 entries (rows = cap / tpk, a multiple
//             of 8).  Key k's entry e belongs to lane ln = (k % K) * tpk + e % tpk as
//             that lane's entry m = e / tpk; each lane's entries sit in 8-entry
//             chunks, chunk c of all 64 lanes side by side, so one 16-byte load per
//             lane reads 8 entries.  Entry = s << 11 | offset: s = stencil cell of
//             the partner (z-major over offsets (ox, oy, oz) in {-1,0,1}^3, 0..26)
//             and the partner's rank within that cell (cells hold at most 2048).
//             Row-tile format (FP32-mixed, one lane per key): entry = 12 * the
//             partner's index in its key's staged row tile (below): the LDS byte
//             offset of its 12-byte record.
//   cells     per box ncell counters and starts, box ranges aligned to 1024-cell tiles.
//   row tiles (FP32-mixed path) each row of cells (fixed cy, cz) is cut into runs of
//             consecutive cells [xa, xb) holding at most kt keys whose staged partner
//             region fits scap records.  The region is the 9 rows (cy+dy, cz+dz),
//             dy, dz in {-1,0,1}, over the unwrapped cells xa-1 .. xb; a row's run is
//             one contiguous range of slots, plus one wrapped cell at either x end
//             ("pieces": row r = (dz+1)*3 + (dy+1), side 0 = cell x = -1, 1 = the
//             run inside [0, n), 2 = cell x = n).  Staged index order: piece by piece,
//             slots in order, so every cell's members are consecutive.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mdg {

constexpr int kWave = 64;
constexpr int kBlock = 256;              // threads per block in every kernel (4 wavefronts)
constexpr int kTile = 1024;              // cells per scan tile
constexpr int kIdxBits = 27;
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;
constexpr int kMaxSeries = 4096;         // energy samples kept per box
constexpr int kMaxCellsPerAxis = 1023;   // 10-bit packed cell coordinates
constexpr int kUnitBits = 28;            // fixed-point units per cell side: at most 2^28
constexpr int kUnitClamp = 1 << 29;      // |u| bound (two cell sides): pair sums stay in int32
constexpr int kOffBits = 11;             // list entry: partner rank within its cell
constexpr int kMaxCellCount = 1 << kOffBits;
constexpr int kStripes = 1024;           // slots per box for per-step maxima
constexpr int kStripeStride = 16;        // 128 bytes between slots
constexpr int kTileWMax = 64;            // cells per row tile at most
constexpr int kScapMax = 5461;           // staged records per row tile at most (16-bit entries of 12 * index)
constexpr int kRtBlock = 256;            // threads per block of the row-tile force kernel (keys per tile)
constexpr int kStageCap = 2432;          // staged records per row tile (28.5 KB of LDS)
constexpr int kRedSeg = 2048;            // energy partials per first-level segment

// Position record of one slot.  cc and cnt ride in the 8 bytes a double4
// would leave unused, so streaming a key's position also brings its cell and
// its list length.
struct __align__(32) Pos {
    double x, y, z;
    uint32_t cc;   // cx | cy << 10 | cz << 20 at the last build
    int32_t cnt;   // list length at the last build
};

struct BoxGeom {
    double L[3];
    double inv[3];   // n / L, rounded once on the host
    double cs[3];    // L / n
    double ucs;      // fixed-point units per length, a power of two with cs * ucs in [2^27, 2^28)
                     // for the largest cell side (the same unit on every axis)
    int32_t uoff[3]; // one cell side in units, per axis: rint(cs * ucs)
    int32_t nuoff[3];// one box length in units modulo 2^32, per axis: n * uoff (the periodic image term)
    float lam;       // length per unit, 1 / ucs (exact)
    float lam2inv;   // ucs^2 (exact)
    float rc2u;      // rc^2 in units^2
    float pad_f;
    int32_t n[3];
    int32_t ncell;
    int32_t cell_off;  // first global cell (multiple of kTile)
    int32_t ntile;
    int32_t tile_off;
    int32_t slot_off;  // first slot (multiple of 64)
    int32_t npart;
    int32_t nslot;
    int32_t id_off;    // first caller index of this box
    int32_t row_off;   // first global row of cells (row = cz * ny + cy within the box)
    // division by d = n[0], n[1], n[0] * n[1] (k = 0, 1, 2) for 0 <= x < 2^30 as
    // (x * dmul[k]) >> (32 + dshr[k]), with dmul = floor(2^(30 + l) / d) + 1 and
    // dshr = l - 2, l = ceil(log2 d): exact over that range, since the multiplier's
    // excess m d - 2^(30 + l) lies in (0, d]
    uint32_t dmul[3];
    int32_t dshr[3];
};

struct BoxState {
    double D;                  // DUTC bound since the last build
    int32_t rebuild;           // list build pending for this box
    int32_t sq;                // current q / u buffer
    int32_t sp;                // current v / id buffer
    int32_t err;               // bit 0: bad position at binning; bit 1: a cell over 2048 particles;
                               // bit 2: a one-cell row tile whose partner region exceeds scap
    int32_t need;              // longest list seen at any build (for overflow detection)
    int32_t built;             // builds done
    unsigned long long missed; // verifier: pairs within rc absent from the list
    double ke, pe;             // last reduced energies
    int32_t nseries;           // energy samples recorded
    int32_t nstep;             // steps opened (drift done, DUTC check run) since the state was set
    double vir;                // last reduced pair virial sum_{i<j} f r^2
    double xi, eta;            // Nose-Hoover thermostat variable and its time integral
    double vscale;             // velocity factor the next kick applies (thermostat; 1 otherwise)
    double thT, thQ;           // thermostat temperature and mass (thQ = 0: no thermostat)
};

struct Params {
    double rc2, rl2, c2, c0, dt, h, mass, skin;  // h = dt / (2 m)
    float rc2f, c2f, c0f, irc2f;  // irc2f: 1 / rc^2 (FP32)
    int32_t cap;        // list entries per key (multiple of 8 * tpk)
    int32_t tpk;        // lanes per key
    int32_t rows;       // cap / tpk, a multiple of 8
    int32_t policy;     // MD_REBUILD_*
    int32_t nbox;
    int32_t nwave;      // 64-slot wavefronts over all boxes
    int32_t ntile;      // cell tiles over all boxes
    int32_t precision;  // MD_PREC_*
    int32_t record;     // energy reduction appends to the series
    int32_t tile;       // row-tile list format and forces from LDS-staged tiles (one lane per key)
    int32_t kt;         // keys per row tile at most (a single cell may hold more)
    int32_t scap;       // staged partner records per row tile at most (LDS: recb bytes each)
    int32_t recb;       // bytes per staged record: 12 (FP32-mixed fixed point), 24 (FP64 x, y, z)
    int32_t tgrid;      // blocks of the row-tile force kernel: one resident round (each loops over tiles)
    int32_t clamp;      // Eq. 1 cutoff (f(rc) = 0): FP32-mixed forces clamp 1/r^2 at 1/rc^2 instead of masking
    int32_t nrows;      // rows of cells over all boxes
    int32_t fastrcp;    // FP64 forces from the hardware reciprocal with the correction of r^-8, r^-14
    int32_t half;       // half list (each pair once, forward stencil cells), partner forces by atomics
    int32_t maxslot;    // slots of the largest box
    int32_t maxcell;    // cells of the largest box
    int32_t redcap;     // first-level energy sums per box (enough for 8 lanes per key)
};

struct Dev {
    BoxGeom* geom;
    BoxState* st;
    int32_t* any;        // nonzero while some box has a list build pending this step
    int32_t* halt;       // nonzero after a list build overflowed (list capacity or a row tile's
                         // staging capacity): the kernels of a step return at once until the
                         // host has grown the list or changed its format and cleared it
    int32_t* wave_box;   // box of each 64-slot wavefront
    int32_t* tile_box;   // box of each cell tile
    Pos* q[2];
    int32_t* u[2];       // fixed-point positions, 3 ints per slot (U3 records)
    double* vx[2];
    double* vy[2];
    double* vz[2];
    int32_t* id[2];
    double4* qb;         // positions at the last build (displacement policy only)
    double* fx;
    double* fy;
    double* fz;
    int32_t* cnt;        // list length per slot
    uint16_t* list;
    int32_t* cell_tmp;   // cell of each (old) slot at binning
    int32_t* ticket;     // arrival rank within the cell at binning
    int32_t* perm;       // new slot -> old slot
    int32_t* cell_cnt;
    int32_t* cell_start;
    int32_t* tile_sum;
    int32_t* tile_pref;
    int32_t* tile_need;  // longest list per cell tile at the last build
    int4* rtile;         // row tiles: (box, row cz * ny + cy, xa, xb), in global row order
    int32_t* row_box;    // box of each global row
    int32_t* row_nt;     // row tiles per row
    int32_t* row_t0;     // first row tile of each row (exclusive scan of row_nt)
    int32_t* ntiles;     // [0] row tiles in all, [1] blocks of the post-build kernel done (the last resets it)
    int32_t* box_t0;     // [nbox + 1] first row tile of each box, then the total
    int32_t* cell_rt;    // row tile of each cell
    int32_t* rt_tmp;     // per cell: xa | xb << 16 of the row's k-th tile at (row's first cell + k)
    int32_t* rt_delta;   // [tile][27]: staged index minus first slot of each piece of the tile
    unsigned long long* vmax_s;  // [nbox][kStripes] striped max |v|^2 (bits), stride kStripeStride
    unsigned long long* disp_s;  // [nbox][kStripes] striped max |q - q_build|^2 (bits)
    double* ke_part;     // per list wave
    double* pe_part;
    double* vir_part;
    double* red;         // [nbox][redcap][3] first-level sums of the ke, pe, vir partials
    double4* dshift;     // [nbox][27] FP64 image shift s * L
    double* series_ke;   // [kMaxSeries][nbox]
    double* series_pe;
    double* series_vir;  // pair virial sum_{i<j} f r^2 at each sample
    double* series_th;   // thermostat share Q xi^2 / 2 + g T eta at each sample
};

// Wrap one coordinate into [0, L) and return its cell index, exactly as the
// plain definition: "if (x < 0) x += L; if (x >= L) x -= L;" then
// min((int)(x * n/L), n - 1).  One IEEE operation per line, no contraction.
__device__ __forceinline__ int bin_axis(double& x, double L, double inv, int n, bool& bad) {
#pragma clang fp contract(off)
    if (!(x >= -L && x < 2.0 * L)) {  // also catches NaN
        bad = true;
        return 0;
    }
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    const double t = x * inv;
    const int k = (int)t;
    return k > n - 1 ? n - 1 : k;
}

// Kernel modes of the force pass.
enum ForceMode : int {
    kForceOnly = 0,  // F -> fx/fy/fz
    kForceEnd = 1,   // v += h F (closing half kick), F stored
    kForceMid = 2    // v += h F twice (close step n, open step n+1), drift q, DUTC max
};

// Subcell grid of the bubble analysis (md_bubbles.hip): n = floor(L / side)
// per axis, inv = n / L rounded once on the host, thr = rho_gas * subcell volume.
struct SubGrid {
    double L[3];
    double inv[3];
    double thr;
    int32_t n[3];
    int32_t nsub;
};

// Device work buffers of the bubble analysis, nsub entries each (flag: 2 ints,
// [0] bad position, [1] root count; cleared by the caller).
struct BubbleWork {
    uint32_t* cnt;   // particles per subcell (cleared by the caller)
    int32_t* par;    // union-find parent, -1 for liquid
    int32_t* lab;    // bubble label (smallest subcell index), -1 for liquid
    int32_t* size;   // subcells per bubble, at its root
    int2* roots;     // (root, size) of each bubble, unordered
    int32_t* flag;
};

void launch_bubbles(const Dev& d, int32_t b, int32_t npart, const SubGrid& sg, const BubbleWork& w, uint8_t* bytes,
                    hipStream_t s);

// Allocation-free bubble analysis: every work buffer lives in a fixed device
// array of the library (md_bubbles.hip), sized for kNaMaxSub subcells.
constexpr int32_t kNaMaxSub = 1 << 20;        // subcells per call at most
constexpr int32_t kNaSeg = 2048;              // subcells per segment of the ordered compaction
constexpr int32_t kNaSegs = kNaMaxSub / kNaSeg;
struct NaMisc {
    int32_t bad;               // a position was not finite or outside [-L, 2L)
    int32_t nroots;            // bubbles found
    unsigned long long ngas;   // gas subcells
    int32_t largest;           // subcells of the largest bubble
    int32_t pad;
};
// Takes the array's device address on `device` (which must be current) once and
// keeps it; later calls return at once.
hipError_t bubbles_scratch_init(int device);
// That address, or nullptr if bubbles_scratch_init has not succeeded on `device`.
unsigned char* bubbles_scratch(int device);
void launch_bubbles_scratch(const Dev& d, int32_t b, int32_t npart, const SubGrid& sg, unsigned char* base,
                            uint8_t* bytes, hipStream_t s);
// Where the results sit inside the array at `base` (device addresses).
void bubbles_scratch_results(unsigned char* base, int64_t** root, int64_t** rsize, int32_t** lab, NaMisc** misc);

// Host-side launchers (md_kernels.hip).  All take the stream to launch on.
void launch_set_state(const Dev& d, const Params& p, const double* pos, const double* vel,
                      int32_t nwave, hipStream_t s);
void launch_get_state(const Dev& d, const Params& p, double* pos, double* vel, int32_t nwave,
                      hipStream_t s);
void launch_get_forces(const Dev& d, const Params& p, double* force, int32_t nwave, hipStream_t s);
void launch_get_cells(const Dev& d, const Params& p, int32_t* cells, int32_t nwave, hipStream_t s);
void launch_list_counts(const Dev& d, const Params& p, int64_t* cnt_by_id, int32_t nwave,
                        hipStream_t s);
void launch_list_export(const Dev& d, const Params& p, const int64_t* key_ptr, int32_t* partners,
                        int32_t nwave, hipStream_t s);
void launch_mark_rebuild(const Dev& d, const Params& p, hipStream_t s);
// Row tiles of every box from the current cell counts (after binning and scans).
void launch_row_tiles(const Dev& d, const Params& p, hipStream_t s);
// Resident blocks per compute unit of the row-tile force kernel.
int rowtile_blocks_per_cu(const Params& p);
void launch_rebuild_chain(const Dev& d, const Params& p, bool with_list, hipStream_t s);
void launch_force(const Dev& d, const Params& p, int mode, bool energy, hipStream_t s);
void launch_kick_drift(const Dev& d, const Params& p, hipStream_t s);
void launch_dutc(const Dev& d, const Params& p, hipStream_t s);
// thermo: bit 0 applies the thermostat half step that ends a step (after the
// closing kick), bit 1 the one that starts the next step; the velocity factor
// goes to BoxState::vscale for the next kick (or k_vscale).
// tl: the partials are per row tile (written by the row-tile force kernel), else per
// list wavefront.
void launch_energy_reduce(const Dev& d, const Params& p, bool record, int thermo, bool tl, hipStream_t s);
void launch_ke_partial(const Dev& d, const Params& p, hipStream_t s);
void launch_vscale(const Dev& d, const Params& p, hipStream_t s);
void launch_verify(const Dev& d, const Params& p, hipStream_t s);
void launch_scale(const Dev& d, const Params& p, const double* alpha_q, const double* scale_v,
                  hipStream_t s);
void launch_list_relayout(const Dev& d, const Params& p, const uint16_t* old, int32_t old_rows, hipStream_t s);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

}  // namespace mdg
