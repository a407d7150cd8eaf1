// Host side of the EPIC/MOFF library: argument validation, FP64 geometry,
// gather lists, device allocation and the extern "C" entry points of
// include/epic.h.  Built with -ffp-contract=off: the nearest-cell indices must
// be bit-identical to an FP64 evaluation of the documented formula.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "epic_gather.hpp"
#include "epic_internal.hpp"
#include "epic_sched.hpp"

using namespace epic;

namespace {

constexpr double kC0 = 299792458.0;   // m/s
constexpr uint32_t kMagic = 0x45504943u;  // 'EPIC'
constexpr uint32_t kKnownFlags = EPIC_F_GRAPH | EPIC_F_AUTOTUNE | EPIC_F_DRY_RUN | EPIC_F_REMOVE_AUTOCORR |
                                 EPIC_F_COMPLEX_WEIGHTS | EPIC_F_ONE_LAUNCH;

// ---- static scratch of epic_image_noalloc ----------------------------------
// Partial accumulators of the allocation-free entry point live in this
// file-scope device array (EPIC_NOALLOC_MAX_BYTES per GPU, held from module
// load to process end) instead of plan-owned memory.  Host code never uses the
// array's name as an address: its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device at plan set-up with that device
// current.
constexpr size_t kNoAllocFloats = (size_t)EPIC_NOALLOC_MAX_BYTES / sizeof(float);
static __device__ __align__(256) float scratch[kNoAllocFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current); looked up
// once per device.
hipError_t scratch_address(int device, float** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<float*>(ptr);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

struct SubHost {
    epic_array_desc desc{};
    std::vector<double> ant_xy;      // [A][2]
    std::vector<float> user_taps;    // [C][A][P][K][K][2] or empty
    std::vector<int32_t> cells;      // [C][A][2]
    std::vector<double> gfrac;       // [C][A][2]
    std::vector<ChanInfo> chans;     // [C]
    std::vector<CellDesc> cells_desc;
    std::vector<uint16_t> grp_ant;
    std::vector<uint8_t> grp_tap;
    // gridding on the matrix cores
    std::vector<BgChan> bg_chans;
    std::vector<uint2> bg_tiles;
    std::vector<uint16_t> bg_cells;
    std::vector<uint16_t> bg_ents;
    std::vector<int32_t> bg_perm;
    std::vector<int32_t> bg_dst;
    // autotuner candidates of this sub-array's launch (gridding form, gather
    // program placement, spectra per gridding step); cands[0] the default
    bool tune = false;
    std::vector<SubDev> cands;
    SubDev dev{};
};

}  // namespace

struct epic_plan_s {
    uint32_t magic = kMagic;
    epic_plan_desc desc{};
    std::vector<SubHost> subs;
    int dry_run = 0;
    int device = 0;
    int num_cu = 256;
    epic_status sticky = EPIC_OK;
    std::vector<void*> allocations;
    int64_t device_bytes = 0;
    // several FP16 sub-arrays: one persistent launch for all of them (batched)
    // or one dedicated launch each; can_batch says the first form exists
    int can_batch = 0;
    int batched = 0;
    double form_ms[2] = {0.0, 0.0};   // autotuner: batched / dedicated call time
    std::vector<SubDev> bdev;        // per sub-array: the batched form's launch shape
    BatchDev bd{};
    std::vector<int> weights;        // cost of one spectrum per sub-array
    std::vector<BatchSub> table;     // host copy of bd.table
    int autotuned = 0;               // 1: timed at plan time, 2: taken from the tuning cache
    // the partial-accumulator slots hold zeros (after plan creation and after a
    // resetting read-out): the next accumulate call stores its sums instead of
    // adding them, which saves reading the slots
    int slots_zero = 1;
    // hipGraph replay of accumulate steps: one executable graph per (spectra
    // count, input pointers), the kGraphCache most recently used kept
    hipStream_t cap_stream = nullptr;
    struct GraphEntry {
        int64_t T;
        int fresh;
        std::vector<const uint8_t*> ptrs;
        hipGraph_t graph;
        hipGraphExec_t exec;
        uint64_t last;
    };
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;
    int graph_builds = 0;
    // autocorrelation removal: spectra in each sub-array's zero-lag sums since
    // their last fold, and the count at which they are folded first
    std::vector<int64_t> ac_pending;
    int64_t ac_limit = 0;
    // host staging of epic_set_gains (pinned, reused once its copy is done)
    float* gain_stage = nullptr;
    size_t gain_stage_n = 0;
    hipEvent_t gain_ev = nullptr;
    int gain_ev_pending = 0;
};

namespace {

bool finite(double v) { return std::isfinite(v); }

epic_status validate_sub(const epic_array_desc& s) {
    if (s.n_ant < 1 || (s.n_pol != 1 && s.n_pol != 2) || s.n_chan < 1) return EPIC_E_ARG;
    if ((int64_t)s.n_ant * s.n_pol > 65536) return EPIC_E_ARG;
    if (s.grid_n < 16 || s.grid_n > kMaxGridN || (s.grid_n % 16) != 0) return EPIC_E_ARG;
    if (s.kernel_k < 1 || s.kernel_k > 7 || (s.kernel_k & 1) == 0) return EPIC_E_ARG;
    if (s.nibble_order != 0 && s.nibble_order != 1) return EPIC_E_ARG;
    if (!finite(s.grid_dl) || !(s.grid_dl > 0.0)) return EPIC_E_ARG;
    if (!finite(s.freq0_hz) || !(s.freq0_hz > 0.0)) return EPIC_E_ARG;
    if (!finite(s.dfreq_hz) || s.dfreq_hz < 0.0) return EPIC_E_ARG;
    if (!s.ant_xy_m) return EPIC_E_ARG;
    if (!finite(s.kernel_sigma_cells)) return EPIC_E_ARG;
    for (int64_t k = 0; k < 2LL * s.n_ant; ++k)
        if (!finite(s.ant_xy_m[k])) return EPIC_E_ARG;
    if (s.taps) {
        int64_t n = (int64_t)s.n_chan * s.n_ant * s.n_pol * s.kernel_k * s.kernel_k * 2;
        for (int64_t k = 0; k < n; ++k)
            if (!std::isfinite(s.taps[k])) return EPIC_E_ARG;
    }
    // entry counts must fit the 32-bit tables
    if ((int64_t)s.n_chan * s.n_ant * s.kernel_k * s.kernel_k > (int64_t)std::numeric_limits<int32_t>::max())
        return EPIC_E_NOMEM;
    return EPIC_OK;
}

// Nearest-cell geometry, Sec. 3.1.  The operation order is part of the ABI.
epic_status geometry(SubHost& h) {
    const epic_array_desc& s = h.desc;
    const int A = s.n_ant, C = s.n_chan, N = s.grid_n, hk = s.kernel_k / 2;
    h.cells.assign((size_t)C * A * 2, 0);
    h.gfrac.assign((size_t)C * A * 2, 0.0);
    for (int c = 0; c < C; ++c) {
        double f = s.freq0_hz + (double)c * s.dfreq_hz;
        for (int a = 0; a < A; ++a)
            for (int ax = 0; ax < 2; ++ax) {
                double u = h.ant_xy[2 * a + ax] * f / kC0;
                double g = u / s.grid_dl + 0.5 * (double)N;
                double p = std::floor(g + 0.5);
                if (!(p - hk >= 0.0) || !(p + hk <= (double)(N - 1))) return EPIC_E_GEOMETRY;
                size_t o = ((size_t)c * A + a) * 2 + ax;
                h.gfrac[o] = g;
                h.cells[o] = (int32_t)p;
            }
    }
    return EPIC_OK;
}

// Per-channel aperture window and gather program: for every non-empty window
// cell, the (antenna, tap) pairs whose kernel footprint covers it, in antenna
// order, padded to whole groups; cells sorted by group count (descending).
void build_gather(SubHost& h) {
    const epic_array_desc& s = h.desc;
    const int A = s.n_ant, C = s.n_chan, K = s.kernel_k, hk = K / 2;
    h.chans.assign(C, ChanInfo{});
    int Rmax = 0, Wmax = 0;
    for (int c = 0; c < C; ++c) {
        const int32_t* cc = &h.cells[(size_t)c * A * 2];
        int x0 = cc[0], x1 = cc[0], y0 = cc[1], y1 = cc[1];
        for (int a = 1; a < A; ++a) {
            x0 = std::min(x0, cc[2 * a]); x1 = std::max(x1, cc[2 * a]);
            y0 = std::min(y0, cc[2 * a + 1]); y1 = std::max(y1, cc[2 * a + 1]);
        }
        ChanInfo& ci = h.chans[c];
        ci.x0 = x0 - hk; ci.y0 = y0 - hk;
        ci.W = x1 - x0 + 1 + 2 * hk; ci.R = y1 - y0 + 1 + 2 * hk;
        Rmax = std::max(Rmax, ci.R); Wmax = std::max(Wmax, ci.W);
    }
    // the transform folds read whole blocks of 8, so the LDS window holds
    // zero-padded rows / columns up to the next multiple of 8
    Rmax = (Rmax + 7) / 8 * 8;
    Wmax = (Wmax + 7) / 8 * 8;
    const int WP = Wmax | 1;   // odd LDS pitch against bank conflicts
    h.dev.Rmax = Rmax; h.dev.Wmax = Wmax; h.dev.WP = WP;
    h.cells_desc.clear(); h.grp_ant.clear(); h.grp_tap.clear();
    int Gmax = 0, CellMax = 0;
    std::vector<std::vector<std::pair<uint16_t, uint8_t>>> lists;
    std::vector<int> order;
    for (int c = 0; c < C; ++c) {
        ChanInfo& ci = h.chans[c];
        const int32_t* cc = &h.cells[(size_t)c * A * 2];
        lists.assign((size_t)ci.R * ci.W, {});
        for (int a = 0; a < A; ++a)
            for (int dy = -hk; dy <= hk; ++dy)
                for (int dx = -hk; dx <= hk; ++dx) {
                    int w = cc[2 * a] + dx - ci.x0, r = cc[2 * a + 1] + dy - ci.y0;
                    lists[(size_t)r * ci.W + w].push_back({(uint16_t)a, (uint8_t)((dy + hk) * K + (dx + hk))});
                }
        order.clear();
        for (int k = 0; k < ci.R * ci.W; ++k)
            if (!lists[k].empty()) order.push_back(k);
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return lists[x].size() > lists[y].size(); });
        ci.n_cell = (int32_t)order.size();
        ci.cell_off = (int32_t)h.cells_desc.size();
        ci.grp_off = (int32_t)(h.grp_ant.size() / kGroup);
        uint32_t g = 0;
        for (int k : order) {
            const auto& L = lists[k];
            const uint32_t ng = (uint32_t)((L.size() + kGroup - 1) / kGroup);
            const uint32_t r = (uint32_t)(k / ci.W), w = (uint32_t)(k % ci.W);
            h.cells_desc.push_back(CellDesc{(r * (uint32_t)WP + w) | (ng << 16), g});
            for (uint32_t e = 0; e < ng * kGroup; ++e) {
                if (e < L.size()) { h.grp_ant.push_back(L[e].first); h.grp_tap.push_back(L[e].second); }
                else { h.grp_ant.push_back(0); h.grp_tap.push_back(255); }
            }
            g += ng;
        }
        ci.n_grp = (int32_t)g;
        Gmax = std::max(Gmax, ci.n_grp);
        CellMax = std::max(CellMax, ci.n_cell);
    }
    h.dev.Gmax = Gmax; h.dev.CellMax = CellMax;
    int r4 = 0;
    for (const ChanInfo& ci : h.chans) r4 = std::max(r4, (ci.R + 3) & ~3);
    h.dev.R4max = r4;
}

// Tables of the GEMM-gridding form (gridding as the product of each channel's
// kernel matrix with the fields, Eq. 4).  Antennas are taken in raster order
// of their positions (north, then east; the order of their cells at every
// channel, up to ties), 32 per block; each channel's non-empty window cells,
// in raster order, 16 per tile.  For every tile the antenna blocks it
// multiplies: the ones with a non-zero weight in the tile, or all of them
// (dense).  Every gather entry (cell, antenna, tap) gets the element of the
// operand block that holds its weight: entry e of the channel's block list,
// lane 16 ((s % 32) / 8) + (row of the cell in its tile), position s % 8,
// with s the antenna's raster position (MFMA A-operand layout).
epic_status build_bgemm(SubHost& h, bool dense) {
    const int A = h.desc.n_ant, C = h.desc.n_chan;
    const int WP = h.dev.WP;
    std::vector<int32_t> order(A);
    for (int a = 0; a < A; ++a) order[a] = a;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const double yx = h.ant_xy[2 * x + 1], yy = h.ant_xy[2 * y + 1];
        if (yx != yy) return yx < yy;
        return h.ant_xy[2 * x] < h.ant_xy[2 * y];
    });
    std::vector<int32_t> pos(A);
    for (int s = 0; s < A; ++s) pos[order[s]] = s;
    const int nablk = (A + 31) / 32;
    h.bg_perm = order;
    h.bg_chans.assign(C, BgChan{});
    h.bg_tiles.clear(); h.bg_cells.clear(); h.bg_ents.clear();
    h.bg_dst.assign(h.grp_ant.size(), -1);
    int64_t n_ent = 0;
    std::vector<int> cell_order;
    std::vector<int> blocks;
    for (int c = 0; c < C; ++c) {
        const ChanInfo& ci = h.chans[c];
        BgChan& bc = h.bg_chans[c];
        bc.tile_off = (int32_t)(h.bg_tiles.size());
        bc.ent_off = (int32_t)n_ent;
        cell_order.resize(ci.n_cell);
        for (int k = 0; k < ci.n_cell; ++k) cell_order[k] = k;
        auto offset = [&](int k) { return (int)(h.cells_desc[ci.cell_off + k].x & 0xFFFFu); };
        std::sort(cell_order.begin(), cell_order.end(), [&](int x, int y) { return offset(x) < offset(y); });
        const int n_tile = (ci.n_cell + 15) / 16;
        bc.n_tile = n_tile;
        int ent_in_chan = 0;
        for (int i = 0; i < n_tile; ++i) {
            blocks.clear();
            for (int rt = 0; rt < 16; ++rt) {
                const int kk = 16 * i + rt;
                if (kk >= ci.n_cell) {
                    h.bg_cells.push_back(0xFFFFu);
                    continue;
                }
                const CellDesc d = h.cells_desc[ci.cell_off + cell_order[kk]];
                const int off = (int)(d.x & 0xFFFFu), ng = (int)(d.x >> 16);
                const int r = off / WP, w = off - r * WP;
                if (r > 255 || w > 255) return EPIC_E_UNSUPPORTED;
                h.bg_cells.push_back((uint16_t)((r << 8) | w));
                for (int e = 0; e < ng * kGroup; ++e) {
                    const size_t ge = ((size_t)ci.grp_off + d.y) * kGroup + e;
                    if (h.grp_tap[ge] != 255) blocks.push_back(pos[h.grp_ant[ge]] / 32);
                }
            }
            if (dense) {
                blocks.resize(nablk);
                for (int j = 0; j < nablk; ++j) blocks[j] = j;
            } else {
                std::sort(blocks.begin(), blocks.end());
                blocks.erase(std::unique(blocks.begin(), blocks.end()), blocks.end());
            }
            h.bg_tiles.push_back(make_uint2((uint32_t)ent_in_chan, (uint32_t)blocks.size()));
            for (int j : blocks) h.bg_ents.push_back((uint16_t)j);
            // operand element of every gather entry of the tile's cells
            for (int rt = 0; rt < 16 && 16 * i + rt < ci.n_cell; ++rt) {
                const CellDesc d = h.cells_desc[ci.cell_off + cell_order[16 * i + rt]];
                const int ng = (int)(d.x >> 16);
                for (int e = 0; e < ng * kGroup; ++e) {
                    const size_t ge = ((size_t)ci.grp_off + d.y) * kGroup + e;
                    if (h.grp_tap[ge] == 255) continue;
                    const int sp = pos[h.grp_ant[ge]];
                    const int q = (int)(std::lower_bound(blocks.begin(), blocks.end(), sp / 32) - blocks.begin());
                    const int64_t ent = n_ent + ent_in_chan + q;
                    const int k = sp & 31;
                    const int64_t el = (ent * 64 + 16 * (k >> 3) + rt) * 8 + (k & 7);
                    if (el > (int64_t)std::numeric_limits<int32_t>::max()) return EPIC_E_UNSUPPORTED;
                    h.bg_dst[ge] = (int32_t)el;
                }
            }
            ent_in_chan += (int)blocks.size();
        }
        bc.n_ent = ent_in_chan;
        n_ent += ent_in_chan;
    }
    if (n_ent * 512 > (int64_t)std::numeric_limits<int32_t>::max()) return EPIC_E_UNSUPPORTED;
    h.dev.bg_nablk = nablk;
    h.dev.bg_nentries = (int64_t)h.grp_ant.size();
    h.dev.bg_nent = n_ent;
    return EPIC_OK;
}

epic_status hip_status(hipError_t e) {
    if (e == hipSuccess) return EPIC_OK;
    if (e == hipErrorOutOfMemory) return EPIC_E_NOMEM;
    return EPIC_E_DEVICE;
}

template <typename T>
epic_status dalloc(epic_plan_s* p, T** ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) return EPIC_OK;
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, count * sizeof(T));
    if (e != hipSuccess) return hip_status(e);
    p->allocations.push_back(v);
    p->device_bytes += (int64_t)(count * sizeof(T));
    *ptr = static_cast<T*>(v);
    return EPIC_OK;
}

template <typename T>
epic_status upload(epic_plan_s* p, T** ptr, const std::vector<T>& v, hipStream_t st) {
    epic_status s = dalloc(p, ptr, v.size());
    if (s != EPIC_OK || v.empty()) return s;
    return hip_status(hipMemcpyAsync(*ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

void free_all(epic_plan_s* p) {
    if (!p->dry_run) {
        (void)hipSetDevice(p->device);
        (void)hipDeviceSynchronize();
        if (p->gain_ev) (void)hipEventDestroy(p->gain_ev);
        if (p->gain_stage) (void)hipHostFree(p->gain_stage);
        p->gain_ev = nullptr; p->gain_stage = nullptr;
        for (auto& g : p->graphs) {
            (void)hipGraphExecDestroy(g.exec);
            (void)hipGraphDestroy(g.graph);
        }
        p->graphs.clear();
        if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
        p->cap_stream = nullptr;
        for (void* v : p->allocations) (void)hipFree(v);
    }
    p->allocations.clear();
}

// Gather weight mode of a sub-array: complex when asked for or when any user
// tap is complex; one weight shared by both pols when every X tap equals its
// Y tap (always so for the default Gaussian); else real per pol.
int weight_mode(const SubHost& h, uint32_t flags) {
    if (flags & EPIC_F_COMPLEX_WEIGHTS) return kWComplex;
    for (size_t k = 1; k < h.user_taps.size(); k += 2)
        if (h.user_taps[k] != 0.0f) return kWComplex;
    if (h.desc.n_pol != 2) return kWReal;
    const size_t kk = (size_t)h.desc.kernel_k * h.desc.kernel_k * 2;   // floats per (c, a, p)
    for (size_t base = 0; base < h.user_taps.size(); base += 2 * kk)
        for (size_t k = 0; k < kk; ++k)
            if (h.user_taps[base + k] != h.user_taps[base + kk + k]) return kWReal;
    return kWShared;
}

// Slots per channel.  A launch runs grid_wg persistent workgroups, each taking
// an equal contiguous run of the (channel, spectrum) sequence, so a channel is
// split over at most ceil(grid_wg / channels) + 1 workgroups (and never more
// than it has spectra); each piece adds into its own slot.
int choose_slots(const SubDev& d, int64_t max_time) {
    const int64_t V = (int64_t)d.C * d.KS;
    int64_t S = (d.grid_wg + V - 1) / V + 1;
    S = std::max<int64_t>(1, std::min<int64_t>(S, max_time));
    return (int)S;
}

// Slots a launch of d's form over up to max_time spectra adds into: the
// direct form's are its time chunks.
int slots_for(const SubDev& d, int64_t max_time) {
    if (d.precision != EPIC_FP32 && d.gridder == EPIC_GRID_DIRECT_GEMM)
        return (int)std::max<int64_t>(1, std::min<int64_t>(d.dir_chunks, max_time));
    return choose_slots(d, max_time);
}

// Cost of one spectrum of one virtual channel in the batched launch, from a
// simple model (CU cycles): MFMA instructions of both transform passes at 4
// cycles per CU, and VALU lane operations (products, gathering, decoding) at
// 64 per cycle.  The autotuner replaces it by measured times.
int model_weight(const SubHost& h) {
    const SubDev& d = h.dev;
    const int NK = d.N / d.KS, IT = NK / 16, WAVES = d.N / 16;
    const int R4 = (d.Rmax + 3) & ~3;
    const double mfma = (double)WAVES * IT * d.P * 2.0 * d.KK + std::ceil(d.P * R4 / 16.0) * (2.0 * NK / 16.0) * d.KK;
    const double entries = (double)h.grp_ant.size() / d.C;
    const double valu = 8.0 * d.N * NK + 4.0 * d.P * entries + 2.0 * d.A * d.P;
    return (int)std::lround(4.0 * mfma + valu / 64.0) + 1;
}

// The batched form of a sub-array: its tables and buffers, with the batched
// kernel's launch shape (gather gridding, whatever form its dedicated launch
// was tuned to).
SubDev batch_view(const SubDev& d, const SubDev& shape) {
    SubDev b = d;
    b.gridder = EPIC_GRID_GATHER;
    b.KK = shape.KK;
    b.KS = shape.KS;
    b.threads = shape.threads;
    b.lds_bytes = shape.lds_bytes;
    b.prog_lds = shape.prog_lds;
    b.grid_wg = shape.grid_wg;
    return b;
}

hipError_t launch_one(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st);

// Time of one accumulate call of Tn spectra in either form, on probe inputs
// and scratch slots (milliseconds, best of three after a warm-up call).
epic_status time_forms(epic_plan_s* p, hipStream_t st, int64_t Tn, const std::vector<const uint8_t*>& in,
                       const std::vector<float*>& slots, BatchSub* table, double* t_batch, double* t_sep) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return EPIC_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return EPIC_E_DEVICE; }
    const int n_sub = (int)p->subs.size();
    std::vector<BatchSub> tab(p->table);
    for (int s = 0; s < n_sub; ++s) tab[s].slots = slots[s];
    epic_status rc = EPIC_OK;
    if (hipMemcpyAsync(table, tab.data(), tab.size() * sizeof(BatchSub), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = EPIC_E_DEVICE;
    BatchDev bd = p->bd;
    bd.table = table;
    double best[2] = {1e30, 1e30};
    for (int form = 0; form < 2 && rc == EPIC_OK; ++form) {
        for (int rep = 0; rep < 4 && rc == EPIC_OK; ++rep) {
            float ms = 0.f;
            hipError_t e = hipEventRecord(e0, st);
            if (e == hipSuccess) {
                if (form == 0) {
                    e = launch_batch(bd, in.data(), n_sub, Tn, st);
                } else {
                    for (int s = 0; s < n_sub && e == hipSuccess; ++s) {   // each in its tuned form
                        SubDev d = p->subs[s].dev;
                        d.slots = slots[s];
                        e = launch_one(d, in[s], Tn, st);
                    }
                }
            }
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { rc = EPIC_E_DEVICE; break; }
            if (rep > 0) best[form] = std::min(best[form], (double)ms);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *t_batch = best[0];
    *t_sep = best[1];
    return rc;
}

// Measure each sub-array's time per spectrum in the batched kernel, alone,
// on all-zero input (the work does not depend on the sample values), and use
// the ratios as the cost weights of the work split.  Each probe gives every
// workgroup a few spectra; the time per spectrum is the slope between a
// probe and one twice as long, which removes the launch and tail overheads.
// The probes add into scratch slots, never into the plan's accumulators.
epic_status autotune_batch(epic_plan_s* p, hipStream_t st, bool choose_form) {
    const int n_sub = (int)p->subs.size();
    const int G = p->bd.grid_wg;
    std::vector<double> tau(n_sub, 0.0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return EPIC_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return EPIC_E_DEVICE; }
    epic_status rc = EPIC_OK;
    for (int s = 0; s < n_sub && rc == EPIC_OK; ++s) {
        const SubDev& d = p->subs[s].dev;
        const int64_t V = (int64_t)d.C * d.KS;
        const int64_t T1 = std::max<int64_t>(2, (2 * G + V - 1) / V), T2 = 2 * T1;
        const int64_t S_probe = (G + V - 1) / V + 1;   // slot bound for any call length
        uint8_t* in = nullptr;
        float* slots = nullptr;
        BatchSub* entry = nullptr;
        const size_t in_bytes = (size_t)T2 * d.C * d.A * d.P;
        const size_t slot_bytes = (size_t)S_probe * d.C * d.NPP * d.N * d.N * sizeof(float);
        if (hipMalloc(&in, in_bytes) != hipSuccess || hipMalloc(&slots, slot_bytes) != hipSuccess ||
            hipMalloc(&entry, sizeof(BatchSub)) != hipSuccess) {
            rc = EPIC_E_NOMEM;
        }
        BatchSub probe = p->table[s];
        probe.slots = slots;
        probe.S = (int)S_probe;
        if (rc == EPIC_OK && (hipMemsetAsync(in, 0, in_bytes, st) != hipSuccess ||
                              hipMemsetAsync(slots, 0, slot_bytes, st) != hipSuccess ||
                              hipMemcpyAsync(entry, &probe, sizeof(BatchSub), hipMemcpyHostToDevice, st) != hipSuccess))
            rc = EPIC_E_DEVICE;
        BatchDev one = p->bd;
        one.table = entry;
        const uint8_t* ptr = in;
        double best[2] = {1e30, 1e30};
        for (int rep = 0; rep < 8 && rc == EPIC_OK; ++rep) {
            const int64_t Tn = (rep & 1) ? T2 : T1;
            float ms = 0.f;
            if (hipEventRecord(e0, st) != hipSuccess || launch_batch(one, &ptr, 1, Tn, st) != hipSuccess ||
                hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = EPIC_E_DEVICE;
                break;
            }
            if (rep >= 2) best[rep & 1] = std::min(best[rep & 1], (double)ms);   // the first pair warms up
        }
        if (rc == EPIC_OK) {
            const double slope = (best[1] - best[0]) / (double)(V * (T2 - T1));
            tau[s] = slope > 0.0 ? slope : best[1] / (double)(V * T2);
        }
        (void)hipStreamSynchronize(st);
        if (entry) (void)hipFree(entry);
        if (slots) (void)hipFree(slots);
        if (in) (void)hipFree(in);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != EPIC_OK) return rc;
    const double tmin = *std::min_element(tau.begin(), tau.end());
    for (int s = 0; s < n_sub; ++s)
        p->table[s].weight = p->weights[s] = std::max(1, (int)std::lround(1000.0 * tau[s] / tmin));
    if (hipMemcpyAsync(p->bd.table, p->table.data(), p->table.size() * sizeof(BatchSub), hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return EPIC_E_DEVICE;
    if (choose_form) {
        // the faster of one batched launch and one dedicated launch per
        // sub-array, timed on a call as long as the plan allows (up to 256)
        const int64_t Tn = std::min<int64_t>(p->desc.max_time, 256);
        std::vector<const uint8_t*> in(n_sub, nullptr);
        std::vector<float*> slots(n_sub, nullptr);
        BatchSub* table = nullptr;
        double tb = 0.0, ts = 0.0;
        epic_status r2 = EPIC_OK;
        for (int s = 0; s < n_sub && r2 == EPIC_OK; ++s) {
            const SubDev& d = p->subs[s].dev;
            const size_t ib = (size_t)Tn * d.C * d.A * d.P;
            int64_t S = std::max(slots_for(d, Tn), choose_slots(p->bdev[s], Tn));
            const size_t sb = (size_t)S * d.C * d.NPP * d.N * d.N * sizeof(float);
            uint8_t* x = nullptr;
            if (hipMalloc(&x, ib) != hipSuccess || hipMalloc(&slots[s], sb) != hipSuccess) r2 = EPIC_E_NOMEM;
            in[s] = x;
            if (r2 == EPIC_OK && (hipMemsetAsync(x, 0, ib, st) != hipSuccess ||
                                  hipMemsetAsync(slots[s], 0, sb, st) != hipSuccess))
                r2 = EPIC_E_DEVICE;
        }
        if (r2 == EPIC_OK && hipMalloc(&table, n_sub * sizeof(BatchSub)) != hipSuccess) r2 = EPIC_E_NOMEM;
        if (r2 == EPIC_OK) r2 = time_forms(p, st, Tn, in, slots, table, &tb, &ts);
        (void)hipStreamSynchronize(st);
        for (int s = 0; s < n_sub; ++s) {
            if (in[s]) (void)hipFree(const_cast<uint8_t*>(in[s]));
            if (slots[s]) (void)hipFree(slots[s]);
        }
        if (table) (void)hipFree(table);
        if (r2 != EPIC_OK) return r2;
        p->batched = tb <= ts ? 1 : 0;
        p->form_ms[0] = tb;
        p->form_ms[1] = ts;
    }
    p->autotuned = 1;
    return EPIC_OK;
}

// The hot kernel of one sub-array in its own launch.
hipError_t launch_one(const SubDev& d, const uint8_t* samples, int64_t n_time, hipStream_t st) {
    if (d.precision == EPIC_FP32) return launch_fp32(d, samples, n_time, st);
    if (d.gridder == EPIC_GRID_DIRECT_GEMM) return launch_direct(d, samples, n_time, st);
    if (d.gridder != EPIC_GRID_GATHER) return launch_bgemm(d, samples, n_time, st);
    return launch_mfma(d, samples, n_time, st);
}

// The kernel launches of one accumulate step.
hipError_t launch_step(epic_plan_s* p, const uint8_t* const* d_samples, int64_t n_time, hipStream_t st) {
    if (p->batched) {
        BatchDev bd = p->bd;
        bd.fresh = p->slots_zero;
        hipError_t e = launch_batch(bd, d_samples, (int)p->subs.size(), n_time, st);
        if (e != hipSuccess) return e;
    } else {
        for (size_t k = 0; k < p->subs.size(); ++k) {
            SubDev d = p->subs[k].dev;
            d.fresh = p->slots_zero;
            hipError_t e = launch_one(d, d_samples[k], n_time, st);
            if (e != hipSuccess) return e;
        }
    }
    // zero-lag antenna correlations for the autocorrelation removal at read-out
    for (size_t k = 0; k < p->subs.size(); ++k) {
        const SubDev& d = p->subs[k].dev;
        if (d.vaa) {
            hipError_t e = launch_autocorr(d, d_samples[k], n_time, st);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

// Replay the step from a captured hipGraph.  Each (spectra count, input
// pointers, first call after a reset or not) gets its own executable graph;
// the kGraphCache most recently used are kept, so a caller that rotates over
// a few input buffers replays instead of capturing again.
constexpr size_t kGraphCache = 8;

hipError_t launch_step_graph(epic_plan_s* p, const uint8_t* const* d_samples, int64_t n_time, hipStream_t st) {
    std::vector<const uint8_t*> ptrs(d_samples, d_samples + p->subs.size());
    epic_plan_s::GraphEntry* hit = nullptr;
    for (auto& g : p->graphs)
        if (g.T == n_time && g.fresh == p->slots_zero && g.ptrs == ptrs) hit = &g;
    if (!hit) {
        if (p->graphs.size() >= kGraphCache) {
            auto lru = std::min_element(p->graphs.begin(), p->graphs.end(),
                                        [](const auto& x, const auto& y) { return x.last < y.last; });
            (void)hipGraphExecDestroy(lru->exec);
            (void)hipGraphDestroy(lru->graph);
            p->graphs.erase(lru);
        }
        epic_plan_s::GraphEntry g{n_time, p->slots_zero, ptrs, nullptr, nullptr, 0};
        hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t le = launch_step(p, d_samples, n_time, p->cap_stream);
        e = hipStreamEndCapture(p->cap_stream, &g.graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (g.graph) (void)hipGraphDestroy(g.graph);
            return le != hipSuccess ? le : e;
        }
        e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g.graph);
            return e;
        }
        p->graphs.push_back(g);
        ++p->graph_builds;
        hit = &p->graphs.back();
    }
    hit->last = ++p->graph_clock;
    return hipGraphLaunch(hit->exec, st);
}

// Zero-lag sums about to pass the exact int32 range: fold them into the lag
// accumulator first (outside any captured graph), then count the new call.
hipError_t autocorr_guard(epic_plan_s* p, int64_t n_time, hipStream_t st) {
    for (size_t k = 0; k < p->subs.size(); ++k) {
        const SubDev& d = p->subs[k].dev;
        if (!d.vaa) continue;
        if (p->ac_pending[k] > 0 && p->ac_pending[k] + n_time > p->ac_limit) {
            hipError_t e = launch_autocorr_fold(d, st);
            if (e != hipSuccess) return e;
            p->ac_pending[k] = 0;
        }
        p->ac_pending[k] += n_time;
    }
    return hipSuccess;
}

// ---- autotuner of the launch forms ------------------------------------------
// Launch-shape settings of a candidate (its tables are the sub-array's own).
void apply_config(SubDev& d, const SubDev& c) {
    d.threads = c.threads;
    d.lds_bytes = c.lds_bytes;
    d.grid_wg = c.grid_wg;
    d.prog_lds = c.prog_lds;
    d.gridder = c.gridder;
    d.bg_tb = c.bg_tb;
    d.KS = c.KS;
    d.KK = c.KK;
    d.dir_chunks = c.dir_chunks;
}

std::string cand_name(const SubDev& c) {
    return "g" + std::to_string(c.gridder) + ",tb" + std::to_string(c.gridder == EPIC_GRID_GATHER ? 1 : c.bg_tb) +
           ",prog" + std::to_string(c.prog_lds);
}

// Time every candidate of every sub-array with more than one, alone, on an
// all-zero probe call (the work does not depend on the sample values) of
// min(max_time, 64) spectra into scratch slots; keep the fastest (best of
// three after a warm-up call).
epic_status tune_forms(epic_plan_s* p, hipStream_t st) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return EPIC_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return EPIC_E_DEVICE; }
    epic_status rc = EPIC_OK;
    bool timed = false;
    for (SubHost& h : p->subs) {
        if (h.cands.size() < 2 || rc != EPIC_OK) continue;
        const SubDev& d = h.dev;
        const int64_t Tn = std::min<int64_t>(p->desc.max_time, 64);
        int64_t S = 1;
        for (const SubDev& c : h.cands)
            S = std::max<int64_t>(S, slots_for(c, Tn));
        uint8_t* in = nullptr;
        float* slots = nullptr;
        const size_t in_bytes = (size_t)Tn * d.C * d.A * d.P;
        const size_t slot_bytes = (size_t)S * d.C * d.NPP * d.N * d.N * sizeof(float);
        if (hipMalloc(&in, in_bytes) != hipSuccess || hipMalloc(&slots, slot_bytes) != hipSuccess) rc = EPIC_E_NOMEM;
        if (rc == EPIC_OK && (hipMemsetAsync(in, 0, in_bytes, st) != hipSuccess ||
                              hipMemsetAsync(slots, 0, slot_bytes, st) != hipSuccess))
            rc = EPIC_E_DEVICE;
        size_t best = 0;
        double best_ms = 1e30;
        for (size_t k = 0; k < h.cands.size() && rc == EPIC_OK; ++k) {
            SubDev run = d;
            apply_config(run, h.cands[k]);
            run.slots = slots;
            run.S = (int)S;
            run.vaa = nullptr;
            double ms_k = 1e30;
            for (int rep = 0; rep < 4 && rc == EPIC_OK; ++rep) {
                float ms = 0.f;
                if (hipEventRecord(e0, st) != hipSuccess || launch_one(run, in, Tn, st) != hipSuccess ||
                    hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = EPIC_E_DEVICE;
                    break;
                }
                if (rep > 0) ms_k = std::min(ms_k, (double)ms);
            }
            if (ms_k < best_ms) {
                best_ms = ms_k;
                best = k;
            }
        }
        (void)hipStreamSynchronize(st);
        if (slots) (void)hipFree(slots);
        if (in) (void)hipFree(in);
        if (rc == EPIC_OK) {
            apply_config(h.dev, h.cands[best]);
            timed = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == EPIC_OK && timed) p->autotuned = 1;
    return rc;
}

// Tuning cache: a JSON object in the file named by EPIC_TUNE_CACHE, one entry
// per line, "key": "value", the key naming the device architecture and the
// plan's shapes, the value the choices (per sub-array candidate names; then
// the launch form and cost weights of a multi-sub-array plan).
std::string tune_key(const epic_plan_s* p) {
    std::string k;
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) k += prop.gcnArchName;
    k += "/cu" + std::to_string(p->num_cu) + "/prec" + std::to_string(p->desc.precision) + "/T" +
         std::to_string(p->desc.max_time) + "/f" + std::to_string(p->desc.flags & (EPIC_F_ONE_LAUNCH | EPIC_F_GRAPH));
    for (const SubHost& h : p->subs) {
        const SubDev& d = h.dev;
        k += "/A" + std::to_string(d.A) + "P" + std::to_string(d.P) + "C" + std::to_string(d.C) + "N" +
             std::to_string(d.N) + "K" + std::to_string(d.K) + "w" + std::to_string(d.wmode) + "R" +
             std::to_string(d.Rmax) + "W" + std::to_string(d.Wmax) + "G" + std::to_string(d.Gmax) + "c" +
             std::to_string(d.CellMax) + "e" + std::to_string(h.bg_ents.size());
    }
    return k;
}

std::vector<std::pair<std::string, std::string>> tune_cache_read(const char* path) {
    std::vector<std::pair<std::string, std::string>> out;
    FILE* f = std::fopen(path, "r");
    if (!f) return out;
    char line[4096];
    while (std::fgets(line, sizeof line, f)) {
        // a line "key": "value"[,]
        std::string s(line);
        const size_t a = s.find('"'), b = s.find("\": \"", a + 1);
        if (a == std::string::npos || b == std::string::npos) continue;
        const size_t c = s.find('"', b + 4);
        if (c == std::string::npos) continue;
        out.emplace_back(s.substr(a + 1, b - a - 1), s.substr(b + 4, c - b - 4));
    }
    std::fclose(f);
    return out;
}

bool tune_cache_get(const std::string& key, std::string* val) {
    const char* path = std::getenv("EPIC_TUNE_CACHE");
    if (!path || !*path) return false;
    for (const auto& kv : tune_cache_read(path))
        if (kv.first == key) {
            *val = kv.second;
            return true;
        }
    return false;
}

void tune_cache_put(const std::string& key, const std::string& val) {
    const char* path = std::getenv("EPIC_TUNE_CACHE");
    if (!path || !*path) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    auto all = tune_cache_read(path);
    bool found = false;
    for (auto& kv : all)
        if (kv.first == key) { kv.second = val; found = true; }
    if (!found) all.emplace_back(key, val);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    for (size_t k = 0; k < all.size(); ++k)
        std::fprintf(f, "\"%s\": \"%s\"%s\n", all[k].first.c_str(), all[k].second.c_str(), k + 1 < all.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    (void)std::rename(tmp.c_str(), path);
}

// "<sub 0 choice>;<sub 1 choice>...|batched|w0,w1,..."
std::string tuned_value(const epic_plan_s* p) {
    std::string v;
    for (size_t k = 0; k < p->subs.size(); ++k) v += (k ? ";" : "") + cand_name(p->subs[k].dev);
    v += "|" + std::to_string(p->batched) + "|";
    for (size_t k = 0; k < p->weights.size(); ++k) v += (k ? "," : "") + std::to_string(p->weights[k]);
    return v;
}

// Apply the per-sub-array choices of a cache entry; false (nothing changed)
// unless every choice names one of the sub-array's candidates.
bool apply_cached_forms(epic_plan_s* p, const std::string& val) {
    const std::string forms = val.substr(0, val.find('|'));
    std::vector<std::string> names;
    size_t a = 0;
    while (a <= forms.size()) {
        const size_t b = forms.find(';', a);
        names.push_back(forms.substr(a, b == std::string::npos ? std::string::npos : b - a));
        if (b == std::string::npos) break;
        a = b + 1;
    }
    if (names.size() != p->subs.size()) return false;
    std::vector<const SubDev*> pick(p->subs.size(), nullptr);
    for (size_t k = 0; k < p->subs.size(); ++k) {
        const SubHost& h = p->subs[k];
        if (h.cands.empty()) {
            if (names[k] != cand_name(h.dev)) return false;
            continue;
        }
        for (const SubDev& c : h.cands)
            if (cand_name(c) == names[k]) pick[k] = &c;
        if (!pick[k]) return false;
    }
    for (size_t k = 0; k < p->subs.size(); ++k)
        if (pick[k]) apply_config(p->subs[k].dev, *pick[k]);
    return true;
}

// The launch form and cost weights of a cache entry (multi-sub-array plans).
epic_status apply_cached_batch(epic_plan_s* p, const std::string& val, hipStream_t st) {
    const size_t a = val.find('|');
    const size_t b = a == std::string::npos ? a : val.find('|', a + 1);
    if (b == std::string::npos) return EPIC_OK;
    p->batched = std::atoi(val.substr(a + 1, b - a - 1).c_str()) != 0 ? 1 : 0;
    size_t k = 0, c = b + 1;
    while (c < val.size() && k < p->weights.size()) {
        p->weights[k] = std::max(1, std::atoi(val.c_str() + c));
        p->table[k].weight = p->weights[k];
        const size_t n = val.find(',', c);
        if (n == std::string::npos) break;
        c = n + 1;
        ++k;
    }
    return hip_status(hipMemcpyAsync(p->bd.table, p->table.data(), p->table.size() * sizeof(BatchSub),
                                     hipMemcpyHostToDevice, st));
}

// Spectra after which the zero-lag sums are folded: every term is at most 128
// in magnitude, so int32 sums stay exact below 2^24 spectra.  The environment
// variable EPIC_AUTOCORR_FOLD_LIMIT can lower it (tests use it to fold often).
int64_t autocorr_fold_limit() {
    const int64_t full = (1LL << 24) - 1;
    const char* env = std::getenv("EPIC_AUTOCORR_FOLD_LIMIT");
    if (!env || !*env) return full;
    char* end = nullptr;
    const long long v = std::strtoll(env, &end, 10);
    if (end == env || *end != '\0' || v < 1 || v > full) return full;
    return (int64_t)v;
}

epic_status make_plan(const epic_plan_desc* desc, hipStream_t st, epic_plan_s* p) {
    p->desc = *desc;
    p->desc.sub = nullptr;
    p->dry_run = (desc->flags & EPIC_F_DRY_RUN) ? 1 : 0;
    p->device = desc->device;
    p->subs.resize(desc->n_sub);
    p->ac_pending.assign(desc->n_sub, 0);
    p->ac_limit = autocorr_fold_limit();
    for (int k = 0; k < desc->n_sub; ++k) {
        SubHost& h = p->subs[k];
        h.desc = desc->sub[k];
        h.ant_xy.assign(desc->sub[k].ant_xy_m, desc->sub[k].ant_xy_m + 2 * (size_t)h.desc.n_ant);
        h.desc.ant_xy_m = nullptr;
        if (desc->sub[k].taps) {
            size_t n = (size_t)h.desc.n_chan * h.desc.n_ant * h.desc.n_pol * h.desc.kernel_k * h.desc.kernel_k * 2;
            h.user_taps.assign(desc->sub[k].taps, desc->sub[k].taps + n);
        }
        h.desc.taps = nullptr;
        epic_status s = geometry(h);
        if (s != EPIC_OK) return s;
        build_gather(h);
        // the gather program stores a cell's window offset r * WP + w in 16
        // bits; such windows (~255 x 255 cells) never fit LDS anyway
        if ((int64_t)h.dev.Rmax * h.dev.WP > 65536) return EPIC_E_UNSUPPORTED;
        SubDev& d = h.dev;
        d.A = h.desc.n_ant; d.P = h.desc.n_pol; d.C = h.desc.n_chan; d.N = h.desc.grid_n;
        d.K = h.desc.kernel_k; d.NPP = (d.P == 2) ? 4 : 1; d.nibble_order = h.desc.nibble_order;
        d.wmode = weight_mode(h, desc->flags);
        d.gridder = desc->gridder;
        if (d.gridder == EPIC_GRID_AUTO) d.gridder = desc->precision == EPIC_FP8 ? EPIC_GRID_BLOCK_GEMM : EPIC_GRID_GATHER;
        // with EPIC_F_AUTOTUNE and the library's choice of gridder, FP16 arrays
        // whose weights the matrix-core product takes are timed both ways
        h.tune = desc->gridder == EPIC_GRID_AUTO && desc->precision == EPIC_FP16 && (desc->flags & EPIC_F_AUTOTUNE) &&
                 !(desc->flags & EPIC_F_ONE_LAUNCH) && (d.wmode == kWShared || (d.P == 1 && d.wmode == kWReal));
        if (h.tune) {
            epic_status bs = build_bgemm(h, false);
            if (bs == EPIC_E_UNSUPPORTED) h.tune = false;
            else if (bs != EPIC_OK) return bs;
        }
        if (d.gridder == EPIC_GRID_DENSE_GEMM || d.gridder == EPIC_GRID_BLOCK_GEMM) {
            // real weights shared by both pols (or single pol) only
            if (!(d.wmode == kWShared || (d.P == 1 && d.wmode == kWReal))) return EPIC_E_UNSUPPORTED;
            epic_status bs = build_bgemm(h, d.gridder == EPIC_GRID_DENSE_GEMM);
            if (bs != EPIC_OK) return bs;
        }
    }
    bool any_gemm = false;
    for (const SubHost& h : p->subs) any_gemm = any_gemm || h.dev.gridder != EPIC_GRID_GATHER;
    if (!p->dry_run) {
        hipError_t e = hipSetDevice(p->device);
        if (e != hipSuccess) return EPIC_E_ARG;
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cu > 0)
            p->num_cu = cu;
        // the allocation-free entry point's scratch address on this device
        float* sp = nullptr;
        if ((e = scratch_address(p->device, &sp)) != hipSuccess) return hip_status(e);
    }
    for (SubHost& h : p->subs) h.dev.precision = desc->precision;
    if (desc->precision == EPIC_FP16 && desc->n_sub > 1 && !any_gemm) {
        // the single persistent launch exists when the sub-arrays share a kernel family
        std::vector<SubDev> devs;
        for (SubHost& h : p->subs) devs.push_back(h.dev);
        hipError_t e = batch_configure(devs.data(), (int)devs.size(), p->bd, p->dry_run ? -1 : p->device, p->num_cu);
        if (e == hipSuccess) {
            p->can_batch = 1;
            p->bdev = devs;
        } else if (e != hipErrorNotSupported) {
            return hip_status(e);
        }
        if ((desc->flags & EPIC_F_ONE_LAUNCH) && !p->can_batch) return EPIC_E_UNSUPPORTED;
        p->batched = (desc->flags & EPIC_F_ONE_LAUNCH) ? 1 : 0;
    } else if (desc->flags & EPIC_F_ONE_LAUNCH) {
        return EPIC_E_UNSUPPORTED;
    }
    for (size_t k = 0; k < p->subs.size(); ++k) {
        SubHost& h = p->subs[k];
        SubDev& d = h.dev;
        const int dev_or_none = p->dry_run ? -1 : p->device;
        hipError_t e = (d.precision == EPIC_FP32)                ? fp32_configure(d, dev_or_none, p->num_cu)
                       : (d.gridder == EPIC_GRID_DIRECT_GEMM) ? direct_configure(d, p->num_cu, desc->max_time)
                       : (d.gridder != EPIC_GRID_GATHER)      ? bg_configure(d, dev_or_none, p->num_cu)
                                                              : mfma_configure(d, dev_or_none, p->num_cu);
        if (e == hipErrorNotSupported) return EPIC_E_UNSUPPORTED;
        if (e != hipSuccess) return hip_status(e);
        // autotuner candidates: the other placement of the gather program, and
        // the block-GEMM form at each step size whose LDS fits
        if (h.tune) {
            h.cands.assign(1, d);
            SubDev alt = d;
            if (mfma_configure(alt, dev_or_none, p->num_cu, d.prog_lds ? 0 : 1) == hipSuccess) h.cands.push_back(alt);
            for (int tb = 16 / (2 * d.P); tb >= 1; tb /= 2) {
                SubDev b = d;
                b.gridder = EPIC_GRID_BLOCK_GEMM;
                if (bg_configure(b, dev_or_none, p->num_cu, tb) == hipSuccess) h.cands.push_back(b);
            }
            SubDev dir = d;
            dir.gridder = EPIC_GRID_DIRECT_GEMM;
            if (direct_configure(dir, p->num_cu, desc->max_time) == hipSuccess) h.cands.push_back(dir);
        }
        // slots for whichever form runs (unused ones stay zero); the direct
        // form's are its time chunks
        d.S = slots_for(d, desc->max_time);
        if (p->can_batch) d.S = std::max(d.S, choose_slots(p->bdev[k], desc->max_time));
        for (const SubDev& c : h.cands)
            d.S = std::max(d.S, slots_for(c, desc->max_time));
        p->weights.push_back(p->can_batch ? model_weight(h) : 1);
        // size checks (also in dry run)
        const double slot_bytes = (double)d.S * d.C * d.NPP * d.N * d.N * 4.0;
        if (slot_bytes > 64.0 * (1ull << 30)) return EPIC_E_NOMEM;
    }
    if (p->dry_run) {
        for (SubHost& h : p->subs) {
            const SubDev& d = h.dev;
            p->device_bytes += (int64_t)d.S * d.C * d.NPP * d.N * d.N * 4 + (int64_t)h.grp_ant.size() * (2 + 1 + 8 * d.P) +
                               (int64_t)h.cells_desc.size() * 8 + (int64_t)d.C * d.A * d.P * d.K * d.K * 8 +
                               (int64_t)h.bg_ents.size() * 512 * (d.precision == EPIC_FP8 ? 3 : 4);
        }
        return EPIC_OK;
    }
    for (SubHost& h : p->subs) {
        SubDev& d = h.dev;
        epic_status s;
        if ((s = upload(p, &d.chans, h.chans, st)) != EPIC_OK) return s;
        if ((s = upload(p, &d.cells_desc, h.cells_desc, st)) != EPIC_OK) return s;
        if ((s = upload(p, &d.grp_ant, h.grp_ant, st)) != EPIC_OK) return s;
        if ((s = upload(p, &d.grp_tap, h.grp_tap, st)) != EPIC_OK) return s;
        if ((s = upload(p, &d.cells, h.cells, st)) != EPIC_OK) return s;
        if ((s = upload(p, &d.gfrac, h.gfrac, st)) != EPIC_OK) return s;
        const size_t ntap = (size_t)d.C * d.A * d.P * d.K * d.K * 2;
        if (!h.user_taps.empty()) {
            if ((s = upload(p, &d.taps, h.user_taps, st)) != EPIC_OK) return s;
        } else {
            if ((s = dalloc(p, &d.taps, ntap)) != EPIC_OK) return s;
            if ((s = hip_status(launch_gaussian_taps(d, h.desc.kernel_sigma_cells > 0.0 ? h.desc.kernel_sigma_cells : 0.5, st))) != EPIC_OK)
                return s;
        }
        d.gains = nullptr;
        if ((s = dalloc(p, &d.grp_w, h.grp_ant.size() * 2 * (size_t)d.P)) != EPIC_OK) return s;
        if ((s = dalloc(p, &d.twiddle, (size_t)d.N)) != EPIC_OK) return s;
        const size_t nslot = (size_t)d.S * d.C * d.NPP * d.N * d.N;
        if ((s = dalloc(p, &d.slots, nslot)) != EPIC_OK) return s;
        if ((s = hip_status(hipMemsetAsync(d.slots, 0, nslot * sizeof(float), st))) != EPIC_OK) return s;
        if ((s = hip_status(launch_twiddles(d, st))) != EPIC_OK) return s;
        if (d.precision != EPIC_FP32 && d.KK > 0) {   // the transform matrix of the grid-and-FFT forms
            uint16_t* m = nullptr;
            if ((s = dalloc(p, &m, (size_t)2 * d.N * 32 * d.KK)) != EPIC_OK) return s;
            d.dft16 = m;
            if ((s = hip_status(launch_dft_matrix(d, st))) != EPIC_OK) return s;
        }
        if ((s = hip_status(launch_entry_weights(d, st))) != EPIC_OK) return s;
        bool need_dir = d.gridder == EPIC_GRID_DIRECT_GEMM;
        for (const SubDev& c : h.cands) need_dir = need_dir || c.gridder == EPIC_GRID_DIRECT_GEMM;
        if (need_dir) {
            uint16_t* m = nullptr;
            if ((s = dalloc(p, &m, (size_t)direct_matrix_halfs(d))) != EPIC_OK) return s;
            d.dir_m = m;
            if ((s = hip_status(launch_direct_matrix(d, st))) != EPIC_OK) return s;
        }
        if (d.gridder == EPIC_GRID_DENSE_GEMM || d.gridder == EPIC_GRID_BLOCK_GEMM || h.tune) {
            if ((s = upload(p, &d.bg_chans, h.bg_chans, st)) != EPIC_OK) return s;
            if ((s = upload(p, &d.bg_tiles, h.bg_tiles, st)) != EPIC_OK) return s;
            if ((s = upload(p, &d.bg_cells, h.bg_cells, st)) != EPIC_OK) return s;
            if ((s = upload(p, &d.bg_ents, h.bg_ents, st)) != EPIC_OK) return s;
            if ((s = upload(p, &d.bg_perm, h.bg_perm, st)) != EPIC_OK) return s;
            if ((s = upload(p, &d.bg_dst, h.bg_dst, st)) != EPIC_OK) return s;
            d.bg_nterm = d.precision == EPIC_FP8 ? 3 : 2;
            const size_t wbytes = h.bg_ents.size() * 512 * (d.precision == EPIC_FP8 ? 1 : 2) * d.bg_nterm;
            if ((s = dalloc(p, &d.bg_w, wbytes)) != EPIC_OK) return s;
            if ((s = dalloc(p, &d.bg_scale, (size_t)2)) != EPIC_OK) return s;
            if ((s = hip_status(hipMemsetAsync(d.bg_w, 0, wbytes, st))) != EPIC_OK) return s;
            if ((s = hip_status(hipMemsetAsync(d.bg_scale, 0, 2 * sizeof(float), st))) != EPIC_OK) return s;
            if ((s = hip_status(launch_bg_weights(d, st))) != EPIC_OK) return s;
        }
        if (desc->flags & EPIC_F_REMOVE_AUTOCORR) {
            const size_t nv = (size_t)d.C * d.A * (d.P == 2 ? 4 : 1);
            const size_t nl = (size_t)d.C * (2 * d.K - 1) * (2 * d.K - 1) * (d.P == 2 ? 3 : 1) * 2;
            if ((s = dalloc(p, &d.vaa, nv)) != EPIC_OK) return s;
            if ((s = dalloc(p, &d.lag, nl)) != EPIC_OK) return s;
            if ((s = hip_status(hipMemsetAsync(d.vaa, 0, nv * sizeof(float), st))) != EPIC_OK) return s;
            if ((s = hip_status(hipMemsetAsync(d.lag, 0, nl * sizeof(float), st))) != EPIC_OK) return s;
        }
    }
    // autotuner: each sub-array's launch candidates timed (or their choice taken
    // from the tuning cache); the single launch of several sub-arrays exists
    // only while every one of them runs the gather form
    std::string tune_key_str, cached;
    bool cache_hit = false;
    if (desc->flags & EPIC_F_AUTOTUNE) {
        tune_key_str = tune_key(p);
        cache_hit = tune_cache_get(tune_key_str, &cached) && apply_cached_forms(p, cached);
        if (!cache_hit) {
            epic_status s = tune_forms(p, st);
            if (s != EPIC_OK) return s;
        }
    }
    // the batched launch always grids by gathering; a sub-array whose tuned
    // dedicated form is a GEMM keeps it for the dedicated launches, and the
    // batch autotuner below times the two launch forms as they would run
    if (p->can_batch) {
        // the batched form shares every table and buffer of the dedicated one
        for (size_t k = 0; k < p->subs.size(); ++k) p->bdev[k] = batch_view(p->subs[k].dev, p->bdev[k]);
        p->table.clear();
        for (size_t k = 0; k < p->subs.size(); ++k) p->table.push_back(batch_entry(p->bdev[k], p->weights[k]));
        epic_status s = dalloc(p, &p->bd.table, p->table.size());
        if (s != EPIC_OK) return s;
        if ((s = hip_status(hipMemcpyAsync(p->bd.table, p->table.data(), p->table.size() * sizeof(BatchSub),
                                           hipMemcpyHostToDevice, st))) != EPIC_OK)
            return s;
        if (desc->flags & EPIC_F_AUTOTUNE) {
            if (cache_hit) {
                if ((s = apply_cached_batch(p, cached, st)) != EPIC_OK) return s;
            } else if ((s = autotune_batch(p, st, (desc->flags & EPIC_F_ONE_LAUNCH) == 0)) != EPIC_OK) {
                return s;
            }
        }
    }
    if ((desc->flags & EPIC_F_AUTOTUNE) && !cache_hit) tune_cache_put(tune_key_str, tuned_value(p));
    if (cache_hit) p->autotuned = 2;
    if (desc->flags & EPIC_F_GRAPH) {
        hipError_t e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_status(e);
    }
    return hip_status(hipStreamSynchronize(st));
}

// Live plans; a handle that is not in this set (never created, or already
// destroyed) is rejected instead of being dereferenced.
std::mutex g_live_mu;
std::set<const epic_plan_s*> g_live;

bool valid_plan(epic_plan_t p) {
    if (p == nullptr) return false;
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.count(p) != 0 && p->magic == kMagic;
}

void register_plan(epic_plan_t p) {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(p);
}

void unregister_plan(epic_plan_t p) {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.erase(p);
}

epic_status check_device(epic_plan_s* p, hipError_t e) {
    if (e == hipSuccess) return EPIC_OK;
    p->sticky = EPIC_E_DEVICE;
    return EPIC_E_DEVICE;
}

}  // namespace

extern "C" {

epic_status epic_plan(const epic_plan_desc* desc, void* hip_stream, epic_plan_t* out) {
    if (!out) return EPIC_E_ARG;
    *out = nullptr;
    if (!desc || desc->n_sub < 1 || desc->n_sub > kMaxSub || !desc->sub) return EPIC_E_ARG;
    if (desc->precision < EPIC_FP32 || desc->precision > EPIC_FP8) return EPIC_E_ARG;
    if (desc->gridder < EPIC_GRID_AUTO || desc->gridder > EPIC_GRID_DIRECT_GEMM) return EPIC_E_ARG;
    if (desc->output != EPIC_OUT_POL && desc->output != EPIC_OUT_STOKES) return EPIC_E_ARG;
    if (desc->max_time < 1 || desc->device < 0) return EPIC_E_ARG;
    if (desc->flags & ~kKnownFlags) return EPIC_E_ARG;
    // the zero-lag correlation pass covers 64 spectra per grid row, 65535 rows
    if ((desc->flags & EPIC_F_REMOVE_AUTOCORR) && desc->max_time > 65535LL * 64) return EPIC_E_UNSUPPORTED;
    for (int k = 0; k < 4; ++k)
        if (desc->reserved[k] != 0) return EPIC_E_ARG;
    for (int k = 0; k < desc->n_sub; ++k) {
        epic_status s = validate_sub(desc->sub[k]);
        if (s != EPIC_OK) return s;
        if (desc->output == EPIC_OUT_STOKES && desc->sub[k].n_pol != 2) return EPIC_E_ARG;
    }
    // gridding on the matrix cores needs a matrix-core precision; FP8 exists
    // only as the gridding product's operand type
    const bool gemm = desc->gridder == EPIC_GRID_DENSE_GEMM || desc->gridder == EPIC_GRID_BLOCK_GEMM;
    if (gemm && desc->precision == EPIC_FP32) return EPIC_E_UNSUPPORTED;
    if (desc->gridder == EPIC_GRID_DIRECT_GEMM && desc->precision != EPIC_FP16) return EPIC_E_UNSUPPORTED;
    if (desc->precision == EPIC_FP8 && desc->gridder == EPIC_GRID_GATHER) return EPIC_E_UNSUPPORTED;
    epic_plan_s* p = new (std::nothrow) epic_plan_s();
    if (!p) return EPIC_E_NOMEM;
    epic_status s;
    try {
        s = make_plan(desc, static_cast<hipStream_t>(hip_stream), p);
    } catch (const std::bad_alloc&) {
        s = EPIC_E_NOMEM;
    }
    if (s != EPIC_OK) {
        free_all(p);
        p->magic = 0;
        delete p;
        return s;
    }
    register_plan(p);
    *out = p;
    return EPIC_OK;
}

epic_status epic_grid_fft_accumulate(epic_plan_t p, const uint8_t* const* d_samples, int64_t n_time,
                                     void* hip_stream) {
    if (!valid_plan(p)) return EPIC_E_ARG;
    if (p->dry_run || p->sticky != EPIC_OK) return EPIC_E_STATE;
    if (n_time < 0 || n_time > p->desc.max_time) return EPIC_E_ARG;
    if (n_time == 0) return EPIC_OK;
    if (!d_samples) return EPIC_E_ARG;
    for (size_t k = 0; k < p->subs.size(); ++k)
        if (!d_samples[k]) return EPIC_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(p->device) != hipSuccess) return check_device(p, hipErrorInvalidDevice);
    hipError_t e = autocorr_guard(p, n_time, st);
    if (e == hipSuccess)
        e = (p->desc.flags & EPIC_F_GRAPH) ? launch_step_graph(p, d_samples, n_time, st)
                                           : launch_step(p, d_samples, n_time, st);
    if (e == hipSuccess) p->slots_zero = 0;
    return check_device(p, e);
}

epic_status epic_efield(epic_plan_t p, int32_t sub, const uint8_t* d_samples, int64_t n_time, float* d_out,
                        void* hip_stream) {
    if (!valid_plan(p) || sub < 0 || sub >= (int32_t)p->subs.size()) return EPIC_E_ARG;
    if (p->dry_run || p->sticky != EPIC_OK) return EPIC_E_STATE;
    if (n_time < 0 || n_time > p->desc.max_time) return EPIC_E_ARG;
    if (p->desc.precision != EPIC_FP32) return EPIC_E_UNSUPPORTED;
    if (n_time == 0) return EPIC_OK;
    if (!d_samples || !d_out) return EPIC_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(p->device) != hipSuccess) return check_device(p, hipErrorInvalidDevice);
    return check_device(p, launch_fp32(p->subs[sub].dev, d_samples, n_time, st, d_out));
}

epic_status epic_readout(epic_plan_t p, float* const* d_images, int32_t reset, void* hip_stream) {
    if (!valid_plan(p)) return EPIC_E_ARG;
    if (p->dry_run || p->sticky != EPIC_OK) return EPIC_E_STATE;
    if (!d_images) return EPIC_E_ARG;
    for (size_t k = 0; k < p->subs.size(); ++k)
        if (!d_images[k]) return EPIC_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(p->device) != hipSuccess) return check_device(p, hipErrorInvalidDevice);
    for (size_t k = 0; k < p->subs.size(); ++k) {
        hipError_t e = launch_readout(p->subs[k].dev, d_images[k], p->desc.output == EPIC_OUT_STOKES, reset != 0, st);
        if (e != hipSuccess) return check_device(p, e);
        if (!p->ac_pending.empty()) p->ac_pending[k] = 0;   // the read-out folded them
    }
    if (reset) p->slots_zero = 1;
    return EPIC_OK;
}

epic_status epic_image_noalloc(epic_plan_t p, const uint8_t* const* d_samples, int64_t n_time,
                               float* const* d_images, void* hip_stream) {
    if (!valid_plan(p)) return EPIC_E_ARG;
    if (p->dry_run || p->sticky != EPIC_OK) return EPIC_E_STATE;
    if (n_time < 0 || n_time > p->desc.max_time) return EPIC_E_ARG;
    if (!d_samples || !d_images) return EPIC_E_ARG;
    for (size_t k = 0; k < p->subs.size(); ++k)
        if (!d_images[k] || (n_time > 0 && !d_samples[k])) return EPIC_E_ARG;
    if (p->desc.flags & EPIC_F_REMOVE_AUTOCORR) return EPIC_E_UNSUPPORTED;
    // partial accumulators of this call: each sub-array's slots for n_time
    // spectra in its dedicated launch, packed into the static scratch
    std::vector<SubDev> run(p->subs.size());
    std::vector<size_t> off(p->subs.size());
    size_t need = 0;
    for (size_t k = 0; k < p->subs.size(); ++k) {
        SubDev d = p->subs[k].dev;
        d.S = slots_for(d, std::max<int64_t>(n_time, 1));
        d.vaa = nullptr;
        off[k] = need;
        need += ((size_t)d.S * d.C * d.NPP * d.N * d.N + 63) & ~(size_t)63;   // 256-byte aligned pieces
        run[k] = d;
    }
    if (need > kNoAllocFloats) return EPIC_E_NOMEM;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(p->device) != hipSuccess) return check_device(p, hipErrorInvalidDevice);
    float* base = nullptr;
    hipError_t e = scratch_address(p->device, &base);
    if (e != hipSuccess) return check_device(p, e);
    for (size_t k = 0; k < run.size(); ++k) {
        run[k].slots = base + off[k];
        run[k].fresh = 1;   // cleared just below
    }
    // clear with a fill kernel (no memset node if the caller captures this)
    e = launch_zero(base, (int64_t)need, st);
    for (size_t k = 0; k < run.size() && e == hipSuccess && n_time > 0; ++k) {
        const SubDev& d = run[k];
        e = launch_one(d, d_samples[k], n_time, st);
    }
    for (size_t k = 0; k < run.size() && e == hipSuccess; ++k)
        e = launch_readout(run[k], d_images[k], p->desc.output == EPIC_OUT_STOKES, 0, st);
    return check_device(p, e);
}

epic_status epic_set_gains(epic_plan_t p, int32_t sub, const float* h_gains, void* hip_stream) {
    if (!valid_plan(p) || sub < 0 || sub >= (int32_t)p->subs.size()) return EPIC_E_ARG;
    if (p->dry_run || p->sticky != EPIC_OK) return EPIC_E_STATE;
    SubDev& d = p->subs[sub].dev;
    const size_t n = (size_t)d.C * d.A * d.P * 2;
    if (h_gains) {
        for (size_t k = 0; k < n; ++k)
            if (!std::isfinite(h_gains[k])) return EPIC_E_ARG;
        // real weights take real gains; weights shared by both pols also need
        // equal X and Y gains (else the plan needs EPIC_F_COMPLEX_WEIGHTS)
        if (d.wmode != kWComplex)
            for (size_t k = 1; k < n; k += 2)
                if (h_gains[k] != 0.0f) return EPIC_E_UNSUPPORTED;
        if (d.wmode == kWShared)
            for (size_t k = 0; k < n; k += 4)
                if (h_gains[k] != h_gains[k + 2]) return EPIC_E_UNSUPPORTED;
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(p->device) != hipSuccess) return check_device(p, hipErrorInvalidDevice);
    // the autocorrelations gathered so far belong to the old gains
    hipError_t e = launch_autocorr_fold(d, st);
    if (e != hipSuccess) return check_device(p, e);
    if (!p->ac_pending.empty()) p->ac_pending[sub] = 0;
    if (!h_gains) {
        d.gains = nullptr;
    } else {
        if (!d.gains_buf) {
            epic_status s = dalloc(p, &d.gains_buf, n);
            if (s != EPIC_OK) return s;
        }
        if (!p->gain_ev && hipEventCreateWithFlags(&p->gain_ev, hipEventDisableTiming) != hipSuccess)
            return check_device(p, hipErrorUnknown);
        if (p->gain_ev_pending) {   // the staging buffer is free once its last copy is done
            if (hipEventSynchronize(p->gain_ev) != hipSuccess) return check_device(p, hipErrorUnknown);
            p->gain_ev_pending = 0;
        }
        if (p->gain_stage_n < n) {
            if (p->gain_stage) (void)hipHostFree(p->gain_stage);
            p->gain_stage = nullptr;
            p->gain_stage_n = 0;
            if (hipHostMalloc(reinterpret_cast<void**>(&p->gain_stage), n * sizeof(float), hipHostMallocDefault) !=
                hipSuccess)
                return EPIC_E_NOMEM;
            p->gain_stage_n = n;
        }
        std::memcpy(p->gain_stage, h_gains, n * sizeof(float));
        e = hipMemcpyAsync(d.gains_buf, p->gain_stage, n * sizeof(float), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventRecord(p->gain_ev, st);
        if (e != hipSuccess) return check_device(p, e);
        p->gain_ev_pending = 1;
        d.gains = d.gains_buf;
    }
    e = launch_entry_weights(d, st);
    if (e == hipSuccess && d.bg_w) e = launch_bg_weights(d, st);
    if (e == hipSuccess && d.dir_m) e = launch_direct_matrix(d, st);
    return check_device(p, e);
}

epic_status epic_plan_query(epic_plan_t p, epic_plan_info* info) {
    if (!valid_plan(p) || !info) return EPIC_E_ARG;
    std::memset(info, 0, sizeof(*info));
    info->n_sub = (int32_t)p->subs.size();
    info->precision = p->desc.precision;
    info->gridder = p->desc.gridder;
    info->output = p->desc.output;
    for (size_t k = 0; k < p->subs.size(); ++k) {
        const SubDev& d = p->subs[k].dev;
        info->npp[k] = (p->desc.output == EPIC_OUT_STOKES) ? 4 : d.NPP;
        info->slots[k] = d.S;
        info->window_max[k] = std::max(d.Rmax, d.Wmax);
        const SubDev& run = p->batched ? p->bdev[k] : d;   // the launch shape in use
        info->threads[k] = run.threads;
        info->lds_bytes[k] = (int64_t)run.lds_bytes;
    }
    info->device_bytes = p->device_bytes;
    info->graph = (p->desc.flags & EPIC_F_GRAPH) ? 1 : 0;
    info->autotuned = p->autotuned;
    info->batched = p->batched;
    info->can_batch = p->can_batch;
    info->form_ms[0] = p->form_ms[0];
    info->form_ms[1] = p->form_ms[1];
    for (size_t k = 0; k < p->subs.size(); ++k) {
        info->weight[k] = p->weights[k];
        info->col_split[k] = p->subs[k].dev.KS;
        info->workgroups[k] = p->batched ? p->bdev[k].grid_wg : p->subs[k].dev.grid_wg;
        info->grid_form[k] = (p->subs[k].dev.precision == EPIC_FP32 || p->batched) ? EPIC_GRID_GATHER
                                                                                    : p->subs[k].dev.gridder;
        const SubDev& dk = p->subs[k].dev;
        info->grid_step[k] = dk.gridder == EPIC_GRID_DIRECT_GEMM ? 16 / dk.P
                             : dk.gridder != EPIC_GRID_GATHER    ? dk.bg_tb
                                                                 : 1;
        info->autocorr_pending[k] = (int32_t)p->ac_pending[k];
        info->grid_blocks[k] = (int64_t)p->subs[k].bg_ents.size();
    }
    info->graph_builds = p->graph_builds;
    info->autocorr_fold_limit = (int32_t)p->ac_limit;
    return EPIC_OK;
}

epic_status epic_debug_schedule(epic_plan_t p, int32_t sub, int64_t n_time, int32_t* h_wg, int32_t* h_slot) {
    if (!valid_plan(p) || !h_wg || !h_slot || sub < 0 || sub >= (int32_t)p->subs.size()) return EPIC_E_ARG;
    if (n_time < 1 || n_time > p->desc.max_time) return EPIC_E_ARG;
    const SubDev& d = p->batched ? p->bdev[sub] : p->subs[sub].dev;
    if (d.gridder == EPIC_GRID_DIRECT_GEMM) return EPIC_E_UNSUPPORTED;   // its own (channel, pixel, time) split
    const int KS = d.KS;
    const int64_t n = (int64_t)d.C * KS * n_time;
    std::fill(h_wg, h_wg + n, -1);
    std::fill(h_slot, h_slot + n, -1);
    const int S = p->subs[sub].dev.S;
    // visit one piece (workgroup g, virtual channel v, spectra [t, t + len)) with slot `slot`
    auto piece = [&](int g, int64_t v, int64_t t, int64_t len, int slot) -> bool {
        if (slot < 0 || slot >= S) return false;
        for (int64_t k = v * n_time + t; k < v * n_time + t + len; ++k) {
            if (h_wg[k] != -1) return false;
            h_wg[k] = g;
            h_slot[k] = slot;
        }
        return true;
    };
    const int G = d.grid_wg;
    if (p->batched) {
        // one launch for all sub-arrays: the cost-weighted sequence over virtual channels
        int64_t total = 0;
        for (size_t s = 0; s < p->subs.size(); ++s)
            total += (int64_t)p->bdev[s].C * p->bdev[s].KS * n_time * p->weights[s];
        const int64_t Lc = (total + G - 1) / G;
        for (int g = 0; g < G; ++g) {
            int64_t base = 0;
            for (int s = 0; s < (int)p->subs.size(); ++s) {
                const SubDev& e = p->bdev[s];
                const int64_t items = (int64_t)e.C * e.KS * n_time, w = p->weights[s];
                int64_t k0, k1;
                owned_range(g, Lc, base, w, items, &k0, &k1);
                if (s == sub) {
                    for (int64_t f = k0; f < k1;) {   // the kernels' segment walk
                        const int64_t v = f / n_time, t = f - v * n_time;
                        const int64_t len = std::min(k1 - f, n_time - t);
                        if (!piece(g, v, t, len, slot_of(g, v, t, n_time, base, w, Lc))) return EPIC_E_STATE;
                        f += len;
                    }
                }
                base += items * w;
            }
        }
    } else {
        // one launch for this sub-array: column-part-major split
        const int64_t total = (int64_t)d.C * n_time;
        for (int g = 0; g < G; ++g) {
            const PartSplit ps = part_split(g, G, KS);
            const int64_t L = (total + ps.Gp - 1) / ps.Gp;
            int64_t k0, k1;
            owned_range(ps.gp, L, 0, 1, total, &k0, &k1);
            for (int64_t f = k0; f < k1;) {
                const int64_t c = f / n_time, t = f - c * n_time;
                const int64_t len = std::min(k1 - f, n_time - t);
                if (!piece(g, c * KS + ps.kpart, t, len, slot_of(ps.gp, c, t, n_time, 0, 1, L))) return EPIC_E_STATE;
                f += len;
            }
        }
    }
    for (int64_t k = 0; k < n; ++k)
        if (h_wg[k] < 0) return EPIC_E_STATE;
    return EPIC_OK;
}

epic_status epic_debug_geometry(epic_plan_t p, int32_t sub, int32_t* h_cells) {
    if (!valid_plan(p) || !h_cells || sub < 0 || sub >= (int32_t)p->subs.size()) return EPIC_E_ARG;
    const SubHost& h = p->subs[sub];
    std::memcpy(h_cells, h.cells.data(), h.cells.size() * sizeof(int32_t));
    return EPIC_OK;
}

epic_status epic_debug_unpack(const uint8_t* d_bytes, int64_t n, int32_t nibble_order, float* d_out,
                              void* hip_stream) {
    if (!d_bytes || !d_out || n < 0 || (nibble_order != 0 && nibble_order != 1)) return EPIC_E_ARG;
    if (n == 0) return EPIC_OK;
    hipError_t e = launch_unpack_debug(d_bytes, n, nibble_order, d_out, static_cast<hipStream_t>(hip_stream));
    return e == hipSuccess ? EPIC_OK : EPIC_E_DEVICE;
}

epic_status epic_destroy(epic_plan_t p) {
    if (!p) return EPIC_OK;
    if (!valid_plan(p)) return EPIC_E_ARG;
    unregister_plan(p);
    free_all(p);
    p->magic = 0;
    delete p;
    return EPIC_OK;
}

const char* epic_status_str(epic_status s) {
    switch (s) {
        case EPIC_OK: return "EPIC_OK";
        case EPIC_E_ARG: return "EPIC_E_ARG";
        case EPIC_E_GEOMETRY: return "EPIC_E_GEOMETRY";
        case EPIC_E_NOMEM: return "EPIC_E_NOMEM";
        case EPIC_E_DEVICE: return "EPIC_E_DEVICE";
        case EPIC_E_UNSUPPORTED: return "EPIC_E_UNSUPPORTED";
        case EPIC_E_STATE: return "EPIC_E_STATE";
    }
    return "EPIC_E_UNKNOWN";
}

int32_t epic_abi_version(void) { return EPIC_ABI_VERSION; }

}  // extern "C"
