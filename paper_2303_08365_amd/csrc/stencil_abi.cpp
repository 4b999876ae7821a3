// stencil_abi.cpp -- host side of libstencil.so: argument checks, plans,
// candidate tilings, pass scheduling and the extern "C" entry points
// declared in include/stencil.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/stencil.h"
#include "internal.h"

using namespace st;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace {

thread_local std::string g_last_error;

st_status fail(st_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

st_status hip_fail(hipError_t e, const char* site) {
    return fail(ST_ERR_HIP, "%s: %s (%d)", site, hipGetErrorString(e), static_cast<int>(e));
}

#define ST_HIP(call, site)                       \
    do {                                         \
        hipError_t e_ = (call);                  \
        if (e_ != hipSuccess) return hip_fail(e_, site); \
    } while (0)

// A device is needed for anything that launches.  Asked once per process.
st_status need_device() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    static int count = 0;
    std::call_once(once, [] { err = hipGetDeviceCount(&count); });
    if (err != hipSuccess) return hip_fail(err, "hipGetDeviceCount");
    if (count < 1) return fail(ST_ERR_HIP, "hipGetDeviceCount: no HIP device");
    return ST_OK;
}

// LDS bytes one work-group may use on the current device.
int device_lds_limit() {
    static std::once_flag once;
    static int limit = 65536;
    std::call_once(once, [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            limit = v;
    });
    return limit;
}

// Compute units of the current device (256 on MI355X; assumed when no
// device is present, so plans made on a host without a GPU match).
int device_cus() {
    static std::once_flag once;
    static int cus = 256;
    std::call_once(once, [] {
        int count = 0, dev = 0, v = 0;
        if (hipGetDeviceCount(&count) == hipSuccess && count > 0 && hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
    });
    return cus;
}

bool have_device() {
    static std::once_flag once;
    static bool ok = false;
    std::call_once(once, [] {
        int count = 0;
        ok = hipGetDeviceCount(&count) == hipSuccess && count > 0;
    });
    return ok;
}

// Fraction of the last dispatch round that is busy when `work` equal items
// run on `cap` resident slots.
double round_fill(int64_t work, int64_t cap) {
    if (work <= 0 || cap <= 0) return 1.0;
    const int64_t rounds = (work + cap - 1) / cap;
    return static_cast<double>(work) / static_cast<double>(rounds * cap);
}

// Chunk length along the streamed axis (extent n): each chunk re-streams
// `halo` extra planes/rows, and `per_chunk` work items exist per chunk.  The
// choice maximises (busy fraction of the dispatch rounds)^(1/4) x (useful
// fraction of the streamed planes); ties go to longer chunks.  The damped
// fill term reflects measurement: waves of a partly filled last round run
// faster, so an idle tail costs far less than its share of slots (on 512^3
// FP64 two fused steps, 47-plane chunks (99 % fill, 92 % useful) beat
// 86-plane chunks (72 % fill, 95 % useful) by 3 %).
int64_t pick_chunk(int64_t n, int64_t per_chunk, int64_t cap, int64_t halo, int64_t min_chunk) {
    double best = -1.0;
    int64_t best_chunk = n;
    for (int64_t c = 1; c <= std::min<int64_t>(n, 1024); ++c) {
        const int64_t chunk = (n + c - 1) / c;
        if ((n + chunk - 1) / chunk != c) continue;
        if (chunk < min_chunk && c > 1) break;
        const double useful = static_cast<double>(n) / static_cast<double>(n + c * halo);
        const double score = std::pow(round_fill(per_chunk * c, cap), 0.25) * useful;
        if (score > best + 1e-9) {
            best = score;
            best_chunk = chunk;
        }
    }
    return best_chunk;
}

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st == hipStreamCaptureStatusActive;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

int elem_bytes(int dtype) { return dtype == kF64 ? 8 : (dtype == kF32 ? 4 : 2); }

}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
namespace {

// One tiling candidate of a plan.
struct Candidate {
    int32_t kernel = ST_KERNEL_NAIVE;
    int32_t tb = 1;
    Stream2DKey k2{};
    Stream3DKey k3{};
    int32_t chunk = 0;  // y chunk (2D) or z chunk (3D); 0 = automatic
    int32_t occ = 0;    // resident work-groups per CU (0 = unknown: assume 2)
    int32_t bpipe = 0;  // ST_KERNEL_BOX3D, two steps: 0 = box3d_kernel, v + 1 = boxpipe3d variant v
};

struct BatchGrid {
    int64_t ny, nx;
};

}  // namespace

struct st_plan_s {
    int32_t ndim = 0;
    int64_t shape[3] = {1, 1, 1};  // caller's extents (ndim used)
    int64_t n[3] = {1, 1, 1};      // nz, ny, nx
    int32_t dtype = kF64;
    int32_t bc = kZero;
    uint32_t flags = 0;
    int32_t npoints = 0;
    int32_t off[kMaxPoints][3] = {};  // canonical order, padded to 3D
    int32_t perm[kMaxPoints] = {};    // canonical index -> caller's index
    int32_t radius = 0;
    int32_t cls = kGeneral;
    std::vector<Candidate> cands;
    int32_t sel = 0;
    // Device memory a plan owns is allocated when the plan is made (see
    // plan_buffers), never by a run call.
    void* owned_work = nullptr;   // ST_PLAN_OWN_WORK
    // outflow runs (zero rule): partial sums of one pass (per wave or per
    // work-group), sized for the largest pass of any candidate
    double* flux_part = nullptr;
    int64_t flux_cap = 0;
    // tessellated 2D candidates: the band scratch, sized for the largest pass
    void* tess_buf = nullptr;
    int64_t tess_cap = 0;
    // batch
    bool batch = false;
    std::vector<BatchGrid> grids;
    void* table_dev = nullptr;            // one Stream2DGrid per grid
    std::vector<unsigned char> table_shadow;  // what the device table holds (empty: unknown)
    // Set once a table upload has been recorded into a caller's graph: every
    // replay of that graph rewrites the device table behind the library's
    // back, so from then on the shadow is never trusted and every run uploads.
    bool table_foreign = false;
    // constant-weight adjoint: the plan of the mirrored point list (host only)
    st_plan_s* mirror = nullptr;
    // ST_PLAN_GRAPH: the launches of the last run, captured and instantiated
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint64_t> graph_key;
};

namespace {

int64_t plan_cells(const st_plan_s* p) { return p->n[0] * p->n[1] * p->n[2]; }

// Classify the (canonical) point set.
void classify(st_plan_s* p) {
    int r = 0;
    for (int i = 0; i < p->npoints; ++i)
        for (int d = 0; d < 3; ++d) r = std::max(r, std::abs(p->off[i][d]));
    p->radius = r;
    p->cls = kGeneral;
    if (r == 0) return;
    const int first = 3 - p->ndim;  // first real axis
    auto has = [&](int dz, int dy, int dx) {
        for (int i = 0; i < p->npoints; ++i)
            if (p->off[i][0] == dz && p->off[i][1] == dy && p->off[i][2] == dx) return true;
        return false;
    };
    // star: centre + every axis point up to r, nothing else
    int star_n = 1 + 2 * p->ndim * r;
    if (p->npoints == star_n) {
        bool ok = true;
        for (int a = first; a < 3 && ok; ++a)
            for (int d = 1; d <= r && ok; ++d)
                for (int sg = -1; sg <= 1; sg += 2) {
                    int o[3] = {0, 0, 0};
                    o[a] = sg * d;
                    if (!has(o[0], o[1], o[2])) { ok = false; break; }
                }
        if (ok) { p->cls = kStar; return; }
    }
    int box_n = 1;
    for (int a = 0; a < p->ndim; ++a) box_n *= 2 * r + 1;
    if (p->npoints == box_n) p->cls = kBox;  // points are distinct and within radius r
}

// Geometry of one 2D pass for a grid.
struct Geo2 {
    int32_t hxa, out_w, tiles_x, chunk_y, chunks_y;
    int64_t items;
};

// Resident waves of the 2D kernel (4 independent waves per work-group).
int64_t wave_capacity2(const Candidate& c) { return static_cast<int64_t>(device_cus()) * (c.occ > 0 ? c.occ : 2) * 4; }

bool geo2(const Candidate& c, int64_t ny, int64_t nx, int tb, Geo2& g, int64_t chunk_override = 0) {
    const int vx = c.k2.vx, R = c.k2.radius;
    if (c.k2.tess) {
        // Tessellated along y: chunks without halo rows, at least one band
        // (2R(tb+1) rows) long so the two junction bands of a chunk never
        // meet; the last chunk takes the remainder.  x as for the overlapped
        // tiling (the band stage gets the strips' ring columns with state 0).
        const int64_t band = tess_band_rows(R, tb);
        g.hxa = static_cast<int32_t>(round_up(static_cast<int64_t>(R) * (tb - 1), vx));
        g.out_w = 64 * vx - 2 * g.hxa;
        if (g.out_w <= 0) return false;
        if (c.k2.bc == kPeriodic && ny < band) return false;  // one chunk wraps onto itself
        g.tiles_x = static_cast<int32_t>(ceil_div(nx, g.out_w));
        int64_t chunk = chunk_override > 0 ? chunk_override : c.chunk;
        // the junction's band costs about 4R*tb row transfers (captured
        // states out, then in again) where the overlapped tiling re-reads
        // 2R*tb rows
        if (chunk <= 0) chunk = pick_chunk(ny, g.tiles_x, wave_capacity2(c), 4 * static_cast<int64_t>(R) * tb, band);
        chunk = std::max<int64_t>(chunk, band);
        const int64_t chunks = std::max<int64_t>(1, ny / chunk);
        g.chunk_y = static_cast<int32_t>(ny / chunks);
        g.chunks_y = static_cast<int32_t>(chunks);
        g.items = static_cast<int64_t>(g.tiles_x) * g.chunks_y;
        return g.items < (int64_t(1) << 31);
    }
    g.hxa = static_cast<int32_t>(round_up(static_cast<int64_t>(R) * (tb - 1), vx));
    g.out_w = 64 * vx - 2 * g.hxa;
    if (g.out_w <= 0) return false;
    g.tiles_x = static_cast<int32_t>(ceil_div(nx, g.out_w));
    int64_t chunk = chunk_override > 0 ? chunk_override : c.chunk;
    if (chunk <= 0)
        chunk = pick_chunk(ny, g.tiles_x, wave_capacity2(c), 2 * static_cast<int64_t>(R) * tb,
                           std::max<int64_t>(8, 2 * R * tb));
    chunk = std::min<int64_t>(chunk, ny);
    g.chunk_y = static_cast<int32_t>(chunk);
    g.chunks_y = static_cast<int32_t>(ceil_div(ny, chunk));
    g.items = static_cast<int64_t>(g.tiles_x) * g.chunks_y;
    return true;
}

// Band scratch of one tessellated pass: per row junction (indexed by the
// chunk below it) and strip, the top and pen arrays of 2R(tb+1) rows of
// 64*VX cells and the rows' ring values (64 per row).
int64_t tess_bytes(const Candidate& c, const Geo2& g, int tb, int dtype) {
    return static_cast<int64_t>(g.chunks_y) * g.tiles_x * tess_band_rows(c.k2.radius, tb) * (2 * 64 * c.k2.vx + 64) *
           elem_bytes(dtype);
}

struct Geo1 {
    int32_t halo, out_w;
    int64_t strips;
};

// 1D strips: 64*VX cells per wave, a stale halo of R*tb cells (rounded up to
// whole lanes) at each end; 32-bit byte offsets (grid below 2 GiB).
bool geo1(const st_plan_s* p, int tb, Geo1& g) {
    const int64_t n = p->n[2];
    if (n * elem_bytes(p->dtype) >= (int64_t(1) << 31)) return false;
    g.halo = static_cast<int32_t>(round_up(static_cast<int64_t>(p->radius) * tb, kStream1DVX));
    g.out_w = 64 * kStream1DVX - 2 * g.halo;
    if (g.out_w < kStream1DVX) return false;
    g.strips = ceil_div(n, g.out_w);
    return true;
}

struct GeoB {
    int32_t tiles_x, tiles_y, chunk_z, chunks_z;
};

// 3D boxes: tiles of out_w x h owned cells (the register tile is 64*VX wide;
// with two steps per pass neighbouring tiles overlap by whole lanes), z
// chunks sized to fill the device; 32-bit plane offsets.
bool geob(const st_plan_s* p, const Candidate& c, int tb, GeoB& g) {
    const int64_t* n = p->n;
    if (tb < 1 || tb > 2) return false;
    if (n[1] * n[2] * elem_bytes(p->dtype) >= (int64_t(1) << 31)) return false;
    if (n[0] >= (int64_t(1) << 30) || n[1] >= (int64_t(1) << 30) || n[2] >= (int64_t(1) << 30)) return false;
    if (c.bpipe > 0 && tb == 2) {
        // the partial-sum pipeline: zero rule, whole-vector rows, the grid
        // at least one register tile wide and high; one work-group of 8
        // waves per CU (2 waves per SIMD); 5 planes re-streamed per chunk
        const BoxPipeShape sh = boxpipe3d_shape(p->dtype, c.bpipe - 1);
        if (p->bc != kZero || n[2] < sh.w || n[1] < sh.h || (sh.vx % 2 == 0 && n[2] % sh.vx != 0)) return false;
        g.tiles_x = static_cast<int32_t>(ceil_div(n[2], sh.out_w));
        g.tiles_y = static_cast<int32_t>(ceil_div(n[1], sh.out_h));
        const int64_t per_plane = static_cast<int64_t>(g.tiles_x) * g.tiles_y;
        int64_t chunk = c.chunk;
        if (chunk <= 0) chunk = pick_chunk(n[0], per_plane, static_cast<int64_t>(device_cus()), 5, 8);
        chunk = std::min<int64_t>(chunk, n[0]);
        g.chunk_z = static_cast<int32_t>(chunk);
        g.chunks_z = static_cast<int32_t>(ceil_div(n[0], chunk));
        return per_plane * g.chunks_z < (int64_t(1) << 31);
    }
    const Box3DShape sh = box3d_shape(p->dtype, tb);
    g.tiles_x = static_cast<int32_t>(ceil_div(n[2], sh.out_w));
    g.tiles_y = static_cast<int32_t>(ceil_div(n[1], sh.h));
    const int64_t per_plane = static_cast<int64_t>(g.tiles_x) * g.tiles_y;
    int64_t chunk = c.chunk;
    if (chunk <= 0) chunk = pick_chunk(n[0], per_plane, static_cast<int64_t>(device_cus()) * 4, 2 * tb, 8);
    chunk = std::min<int64_t>(chunk, n[0]);
    g.chunk_z = static_cast<int32_t>(chunk);
    g.chunks_z = static_cast<int32_t>(ceil_div(n[0], chunk));
    return per_plane * g.chunks_z < (int64_t(1) << 31);
}

struct Geo3 {
    int32_t hxa, hya, out_w, out_h, tiles_x, tiles_y, chunk_z, chunks_z;
};

bool geo3(const Candidate& c, const int64_t n[3], int tb, Geo3& g) {
    const int vx = c.k3.vx, R = c.k3.radius, H = c.k3.k * c.k3.nw;
    // the kernel addresses a plane with 32-bit byte offsets and indexes with
    // 32-bit integers: planes below 2 GiB, every extent below 2^30
    if (n[1] * n[2] * elem_bytes(c.k3.dtype) >= (int64_t(1) << 31)) return false;
    if (n[0] >= (int64_t(1) << 30) || n[1] >= (int64_t(1) << 30) || n[2] >= (int64_t(1) << 30)) return false;
    // the queued-plane kernel brings the R columns beyond its register tile
    // to step 0 (x ring); the partial-sum pipeline does not, so its level l
    // is exact l*R columns in from each side
    const int64_t hx = c.k3.pipe ? static_cast<int64_t>(R) * tb : static_cast<int64_t>(R) * (tb - 1);
    g.hxa = static_cast<int32_t>(round_up(hx, vx));
    g.hya = R * (tb - 1);
    g.out_w = 64 * vx - 2 * g.hxa;
    g.out_h = H - 2 * g.hya;
    if (g.out_w <= 0 || g.out_h <= 0) return false;
    g.tiles_x = static_cast<int32_t>(ceil_div(n[2], g.out_w));
    g.tiles_y = static_cast<int32_t>(ceil_div(n[1], g.out_h));
    int64_t chunk = c.chunk;
    const int64_t per_plane = static_cast<int64_t>(g.tiles_x) * g.tiles_y;
    if (chunk <= 0) {
        const int64_t cap = static_cast<int64_t>(device_cus()) * (c.occ > 0 ? c.occ : 2);
        chunk = pick_chunk(n[0], per_plane, cap, 2 * static_cast<int64_t>(R) * tb,
                           std::max<int64_t>(8, 2 * R * tb));
    }
    chunk = std::min<int64_t>(chunk, n[0]);
    g.chunk_z = static_cast<int32_t>(chunk);
    g.chunks_z = static_cast<int32_t>(ceil_div(n[0], chunk));
    return per_plane * g.chunks_z < (int64_t(1) << 31);
}

// Default fused depth and lane width per family.
int default_vx2(int dtype) { return dtype == kF64 ? 2 : (dtype == kF32 ? 4 : 8); }

void build_candidates(st_plan_s* p) {
    p->cands.clear();
    Candidate naive;
    naive.kernel = ST_KERNEL_NAIVE;
    naive.tb = 1;
    if (p->flags & ST_PLAN_VARCOEF) {
        Candidate v;
        v.kernel = ST_KERNEL_VARCOEF3D;
        v.tb = 1;
        p->cands.push_back(v);
        p->sel = 0;
        return;
    }
    const bool force_naive = (p->flags & ST_PLAN_NAIVE) != 0;
    std::vector<Candidate> fast;
    // Chunk lengths along the streamed axis offered to the autotuner besides
    // the model's choice (0): measured optima on MI355X range from 4 rows (a
    // 512^2 grid, latency bound) through 48 (the 64-grid batch) and 95 (8192^2)
    // to 64 planes (512^3).
    const int chunks2[] = {0, 4, 8, 16, 32, 48, 64, 96, 128};
    const int chunks3[] = {0, 32, 64, 128};
    if (!force_naive && p->ndim == 2 && p->radius <= 2 && (p->cls == kStar || p->cls == kBox)) {
        const int vx = default_vx2(p->dtype);
        const int tbs[] = {1, 2, 4, 8};
        for (int ch : chunks2) {
            if (ch > p->n[1]) continue;
            for (int tb : tbs) {
                for (int tbmax : {1, 4, 8}) {
                    if (tbmax < tb) continue;
                    Candidate c;
                    c.kernel = ST_KERNEL_STREAM2D;
                    c.tb = tb;
                    c.chunk = ch;
                    c.k2 = Stream2DKey{p->dtype, p->bc, p->cls, p->radius, tbmax, vx};
                    if (stream2d_has(c.k2) && have_device()) c.occ = stream2d_occupancy(c.k2);
                    Geo2 g;
                    if (stream2d_has(c.k2) && geo2(c, p->n[1], p->n[2], tb, g)) {
                        fast.push_back(c);
                        break;  // smallest instance that holds tb
                    }
                }
            }
        }
        // heuristic default first: deeper fusion for narrower storage, model chunk
        // (radius 2: at most four fused steps are instantiated)
        const int want = (p->dtype == kF64 || p->radius == 2) ? 4 : 8;
        std::stable_sort(fast.begin(), fast.end(), [&](const Candidate& a, const Candidate& b) {
            return (a.tb == want && a.chunk == 0) > (b.tb == want && b.chunk == 0);
        });
        // the tessellated tiling (no recomputed halo rows, a band stage per
        // pass) as further candidates of single-grid plans
        if (!p->batch) {
            for (int tb : {2, 4, 1, 3})
                for (int ch : {0, 64, 128, 256}) {
                    Candidate c;
                    c.kernel = ST_KERNEL_STREAM2D;
                    c.tb = tb;
                    c.chunk = ch;
                    c.k2 = Stream2DKey{p->dtype, p->bc, p->cls, p->radius, 4, vx, 0, 1};
                    if (!stream2d_has(c.k2)) continue;
                    if (ch > 0 && ch >= p->n[1]) continue;
                    if (have_device()) c.occ = stream2d_occupancy(c.k2);
                    Geo2 g;
                    if (geo2(c, p->n[1], p->n[2], tb, g)) fast.push_back(c);
                }
        }
    }
    if (!force_naive && p->ndim == 3 && p->cls == kStar && (p->radius == 1 || p->radius == 4)) {
        // ylds: step-0 y neighbours through LDS, the tile's halo rows loaded once
        struct V { int vx, k, nw, late, ylds, pipe; };
        std::vector<V> vs;
        if (p->radius == 1) {
            // first: the fastest measured on MI355X for 512^3 at the default
            // depth.  The partial-sum pipeline (pipe = NB*10 + PD, +100 for the
            // LDS input queue) at four fused steps: FP64 1075 Gcell/s with two
            // LDS buffers and 4 rows x 128 columns per wave (LDS queue: 955);
            // FP32 1623 with 8 rows x 128 columns (4 rows x 256 columns: 1530,
            // LDS queue 1574); bfloat16 (three steps) 1895 with 6 rows x 256
            // columns (4 rows: 1631).  The queued-plane kernel: 740 / 1394.
            if (p->dtype == kF64)
                vs = {{2, 4, 8, 0, 0, 21}, {2, 4, 8, 0, 0, 112}, {2, 4, 8, 1, 1}, {2, 4, 8, 1, 0},
                      {2, 4, 8, 0, 0},     {2, 4, 4, 0, 0},      {2, 2, 8, 0, 0}, {2, 3, 8, 1, 0},
                      {2, 4, 8, 0, 1},     {2, 5, 8, 1, 1},      {2, 4, 8, 0, 0, 11}, {2, 3, 8, 0, 0, 21}};
            else if (p->dtype == kF32)
                vs = {{2, 8, 8, 0, 0, 21}, {4, 4, 8, 0, 0, 21}, {4, 4, 8, 0, 0, 112}, {4, 4, 8, 1, 1},
                      {4, 4, 8, 1, 0},     {4, 4, 8, 0, 0},     {4, 4, 4, 0, 0},      {4, 2, 8, 0, 0},
                      {4, 3, 8, 1, 0},     {4, 4, 8, 0, 1},     {4, 5, 8, 1, 1},      {4, 4, 8, 0, 0, 11},
                      {4, 3, 8, 0, 0, 21}};
            else
                vs = {{4, 6, 8, 0, 0, 21}, {4, 4, 8, 0, 0, 21}, {4, 4, 8, 0, 1}, {4, 4, 4, 0, 0}};
        } else {
            // radius 4: the y halo through LDS (ylds) loads 2R rows per tile
            // instead of 2R per wave
            if (p->dtype == kF64) vs = {{4, 1, 8, 0, 1}, {4, 1, 8, 0, 0}};
            else if (p->dtype == kF32) vs = {{4, 2, 8, 0, 1}, {4, 1, 16, 0, 1}, {4, 2, 8, 0, 0}, {4, 1, 16, 0, 0}};
            else vs = {{4, 2, 8, 0, 1}, {4, 2, 8, 0, 0}};
        }
        for (int ch : chunks3) {
            if (ch > p->n[0]) continue;
            for (int tb = 1; tb <= 4; ++tb) {
                for (const V& v : vs) {
                    for (int tbmax : {1, 2, 3, 4}) {
                        if (tbmax < tb) continue;
                        Candidate c;
                        c.kernel = ST_KERNEL_STREAM3D;
                        c.tb = tb;
                        c.chunk = ch;
                        c.k3 = Stream3DKey{p->dtype, p->bc, p->radius, tbmax, v.vx, v.k, v.nw, 1, v.late, v.ylds,
                                           0, v.pipe};
                        if (!stream3d_has(c.k3)) continue;
                        // on a device, only tilings whose LDS it can give
                        if (have_device() && stream3d_lds_bytes(c.k3) > device_lds_limit()) continue;
                        if (have_device()) c.occ = stream3d_occupancy(c.k3);
                        Geo3 g;
                        if (geo3(c, p->n, tb, g)) {
                            fast.push_back(c);
                            break;
                        }
                    }
                }
            }
        }
        // measured on MI355X (512^3, radius 1, 100 steps): four fused steps of
        // the pipeline for FP64 and FP32 (1081 and 1625 Gcell/s; three: 913
        // and 1483); bfloat16 three (1895; four: 1488; one step of the
        // queued-plane kernel: 1384)
        const int want = p->radius == 1 ? (p->dtype == kBF16 ? 3 : 4) : 1;
        std::stable_sort(fast.begin(), fast.end(), [&](const Candidate& a, const Candidate& b) {
            return (a.tb == want && a.chunk == 0) > (b.tb == want && b.chunk == 0);
        });
    }
    if (!force_naive && p->ndim == 3 && p->cls == kBox && p->radius == 1) {
        // FP64 under the zero rule: two steps through the partial-sum
        // pipeline first (512^3: 425 against 328 Gcell/s for one step per
        // pass).  Otherwise one step per pass first: the wave-independent
        // two-step variant recomputes 2 of every 4 rows at its first step
        // (266 vs 326 Gcell/s FP64, 408 vs 639 FP32), and the pipeline's FP32
        // and bfloat16 forms are VALU-bound at two steps (633 vs 654, 523 vs
        // 862): without packed math FP32 runs at the FP64 vector rate, so two
        // fused steps cost more than a one-step pass's HBM time; they stay
        // candidates for the autotuner.
        const auto add_pipe = [&]() {
            for (int v = 0; v < boxpipe3d_variants(p->dtype); ++v)
                for (int ch : {0, 16}) {
                    Candidate c;
                    c.kernel = ST_KERNEL_BOX3D;
                    c.tb = 2;
                    c.chunk = ch;
                    c.bpipe = v + 1;
                    GeoB g;
                    if ((ch == 0 || ch < p->n[0]) && geob(p, c, 2, g)) fast.push_back(c);
                }
        };
        if (p->dtype == kF64) add_pipe();
        for (int tb : {1, 2})
            for (int ch : {0, 16, 32, 64}) {
                Candidate c;
                c.kernel = ST_KERNEL_BOX3D;
                c.tb = tb;
                c.chunk = ch;
                GeoB g;
                if ((ch == 0 || ch < p->n[0]) && geob(p, c, tb, g)) fast.push_back(c);
            }
        if (p->dtype != kF64) add_pipe();
    }
    if (!force_naive && p->ndim == 1 && p->cls == kStar && stream1d_has(p->dtype, p->radius)) {
        // the whole space-time tile in registers: any depth; deeper passes
        // trade halo recomputation (2*R*tb of 1024 cells) for HBM passes
        for (int tb : {32, 1, 2, 4, 8, 16, 64, 128}) {
            Candidate c;
            c.kernel = ST_KERNEL_STREAM1D;
            c.tb = tb;
            Geo1 g;
            if (geo1(p, tb, g)) fast.push_back(c);
        }
    }
    // STENCIL_CHUNK: fixed chunk length along the streamed axis (tuning)
    if (const char* ch = std::getenv("STENCIL_CHUNK")) {
        const int v = std::atoi(ch);
        if (v > 0)
            for (Candidate& c : fast) c.chunk = v;
    }
    p->cands = fast;
    p->cands.push_back(naive);
    p->sel = 0;
    // environment overrides (testing and tuning): STENCIL_TB, STENCIL_VARIANT
    if (const char* v = std::getenv("STENCIL_VARIANT")) {
        const int i = std::atoi(v);
        if (i >= 0 && i < static_cast<int>(p->cands.size())) p->sel = i;
    } else if (const char* t = std::getenv("STENCIL_TB")) {
        const int tb = std::atoi(t);
        for (size_t i = 0; i < p->cands.size(); ++i)
            if (p->cands[i].tb == tb) { p->sel = static_cast<int>(i); break; }
    }
}

st_status check_pattern(const st_pattern* pat) {
    if (!pat) return fail(ST_ERR_ARG, "pattern is NULL");
    if (pat->ndim < 1 || pat->ndim > 3) return fail(ST_ERR_UNSUPPORTED, "ndim %d not in 1..3", pat->ndim);
    if (pat->npoints < 1 || pat->npoints > kMaxPoints)
        return fail(pat->npoints < 1 ? ST_ERR_ARG : ST_ERR_UNSUPPORTED, "npoints %d not in 1..%d",
                    pat->npoints, kMaxPoints);
    if (!pat->offsets) return fail(ST_ERR_ARG, "pattern offsets are NULL");
    bool centre = false;
    for (int i = 0; i < pat->npoints; ++i) {
        bool zero = true;
        for (int d = 0; d < pat->ndim; ++d) {
            const int o = pat->offsets[i * pat->ndim + d];
            if (o < -kMaxRadius || o > kMaxRadius)
                return fail(ST_ERR_UNSUPPORTED, "offset %d of point %d exceeds radius %d", o, i, kMaxRadius);
            zero = zero && o == 0;
        }
        centre = centre || zero;
        for (int j = 0; j < i; ++j) {
            bool same = true;
            for (int d = 0; d < pat->ndim; ++d)
                same = same && pat->offsets[i * pat->ndim + d] == pat->offsets[j * pat->ndim + d];
            if (same) return fail(ST_ERR_ARG, "points %d and %d coincide", j, i);
        }
    }
    if (!centre) return fail(ST_ERR_ARG, "the centre point (all offsets 0) is missing");
    return ST_OK;
}

st_status fill_plan(st_plan_s* p, const st_pattern* pat, st_dtype storage, st_boundary bc, uint32_t flags) {
    if (storage != ST_F64 && storage != ST_F32 && storage != ST_BF16)
        return fail(ST_ERR_ARG, "storage dtype %d unknown", static_cast<int>(storage));
    if (bc != ST_BC_ZERO && bc != ST_BC_PERIODIC) return fail(ST_ERR_ARG, "boundary %d unknown", static_cast<int>(bc));
    if (flags & ~(ST_PLAN_AUTOTUNE | ST_PLAN_NAIVE | ST_PLAN_VARCOEF | ST_PLAN_GRAPH | ST_PLAN_OWN_WORK))
        return fail(ST_ERR_ARG, "unknown flag bits 0x%x", flags);
    p->ndim = pat->ndim;
    p->dtype = storage;
    p->bc = bc;
    p->flags = flags;
    p->npoints = pat->npoints;
    // canonical order: centre first, then lexicographic by padded offset
    std::vector<std::array<int, 4>> pts;
    for (int i = 0; i < pat->npoints; ++i) {
        std::array<int, 4> o = {0, 0, 0, i};
        for (int d = 0; d < pat->ndim; ++d) o[3 - pat->ndim + d] = pat->offsets[i * pat->ndim + d];
        pts.push_back(o);
    }
    std::sort(pts.begin(), pts.end(), [](const std::array<int, 4>& a, const std::array<int, 4>& b) {
        const bool ca = a[0] == 0 && a[1] == 0 && a[2] == 0, cb = b[0] == 0 && b[1] == 0 && b[2] == 0;
        if (ca != cb) return ca;
        return std::lexicographical_compare(a.begin(), a.begin() + 3, b.begin(), b.begin() + 3);
    });
    for (int i = 0; i < p->npoints; ++i) {
        for (int d = 0; d < 3; ++d) p->off[i][d] = pts[i][d];
        p->perm[i] = pts[i][3];
    }
    classify(p);
    if (flags & ST_PLAN_VARCOEF) {
        if (p->ndim != 3 || p->cls != kStar || p->radius != 1)
            return fail(ST_ERR_UNSUPPORTED, "variable-coefficient plans take the 3D radius-1 star");
        if (bc != ST_BC_ZERO) return fail(ST_ERR_UNSUPPORTED, "variable-coefficient plans use the zero boundary");
        if (storage == ST_BF16) return fail(ST_ERR_UNSUPPORTED, "variable-coefficient plans store FP64 or FP32");
    }
    return ST_OK;
}

// Weights in canonical order, rounded once to the compute precision.
void canonical_weights(const st_plan_s* p, const double* coeffs, double* out) {
    for (int i = 0; i < p->npoints; ++i) {
        const double w = coeffs[p->perm[i]];
        out[i] = (p->dtype == kF64) ? w : static_cast<double>(static_cast<float>(w));
    }
}

bool aligned16(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15u) == 0; }

// Fused depths of the passes of one run: all tb except the remainder, and
// arranged so that their count is even (the last pass then writes the
// caller's grid).  `copy` is set when that is impossible (every pass is a
// single step and the count is odd).
std::vector<int> pass_list(int64_t steps, int tb, bool& copy) {
    std::vector<int> v;
    copy = false;
    if (steps <= 0) return v;
    for (int64_t s = 0; s + tb <= steps; s += tb) v.push_back(tb);
    if (steps % tb) v.push_back(static_cast<int>(steps % tb));
    if (v.size() % 2 == 1) {
        // split the last pass of depth >= 2 into two
        for (int i = static_cast<int>(v.size()) - 1; i >= 0; --i) {
            if (v[i] >= 2) {
                const int a = v[i] / 2, b = v[i] - a;
                v[i] = a;
                v.insert(v.begin() + i + 1, b);
                return v;
            }
        }
        copy = true;
    }
    return v;
}

// The whole-vector form of a 3D tiling applies to this grid (what
// launch_pass decides per pass from the same facts).
bool fast3(const st_plan_s* p, const Candidate& c, bool vec_ok) {
    return vec_ok && (p->bc == kPeriodic || (p->n[2] >= 64 * c.k3.vx && p->n[1] >= static_cast<int64_t>(c.k3.k) * c.k3.nw));
}

st_status launch_pass(const st_plan_s* p, const Candidate& c, const void* src, void* dst,
                      const double* wcan, int tb, bool vec_ok, hipStream_t s, double* fpart = nullptr) {
    hipError_t e = hipSuccess;
    if (c.kernel == ST_KERNEL_NAIVE) {
        NaiveArgs a;
        a.src = src;
        a.dst = dst;
        for (int d = 0; d < 3; ++d) a.n[d] = p->n[d];
        a.npoints = p->npoints;
        a.bc = p->bc;
        for (int i = 0; i < p->npoints; ++i) {
            for (int d = 0; d < 3; ++d) a.off[i][d] = p->off[i][d];
            a.w[i] = wcan[i];
        }
        for (int t = 0; t < tb && e == hipSuccess; ++t) {
            // tb > 1 never reaches here: the naive family runs single steps
            e = launch_naive(p->dtype, a, s);
        }
        if (e != hipSuccess) return hip_fail(e, "naive launch");
        return ST_OK;
    }
    if (c.kernel == ST_KERNEL_BOX3D) {
        GeoB g;
        // the pipeline takes two-step passes over whole-vector rows; any
        // other pass of the candidate runs on box3d_kernel (same bits)
        Candidate cb = c;
        if (cb.bpipe > 0) {
            const BoxPipeShape sh = boxpipe3d_shape(p->dtype, cb.bpipe - 1);
            const bool ok = tb == 2 && (sh.vx % 2 != 0 || p->n[2] % sh.vx == 0) && aligned16(src) && aligned16(dst);
            if (!ok || !geob(p, cb, tb, g)) {
                cb.bpipe = 0;
                cb.chunk = 0;
            }
        }
        if (!geob(p, cb, tb, g)) return fail(ST_ERR_UNSUPPORTED, "3D box tiling infeasible");
        Box3DArgs a;
        std::memset(&a, 0, sizeof(a));
        a.src = src;
        a.dst = dst;
        a.nz = p->n[0];
        a.ny = p->n[1];
        a.nx = p->n[2];
        a.tiles_x = g.tiles_x;
        a.tiles_y = g.tiles_y;
        a.chunks_z = g.chunks_z;
        a.chunk_z = g.chunk_z;
        a.tb = tb;
        for (int i = 0; i < p->npoints; ++i) a.w[i] = wcan[i];
        if (cb.bpipe > 0) {
            e = launch_boxpipe3d(p->dtype, cb.bpipe - 1, a, s);
            if (e != hipSuccess) return hip_fail(e, "boxpipe3d launch");
            return ST_OK;
        }
        // whole-vector rows; under the zero rule the edge tiles move inward,
        // which needs the grid at least one register tile wide
        const bool fast = vec_ok && (p->bc == kPeriodic || p->n[2] >= box3d_shape(p->dtype, tb).w);
        e = launch_box3d(p->dtype, p->bc == kPeriodic, fast, a, s);
        if (e != hipSuccess) return hip_fail(e, "box3d launch");
        return ST_OK;
    }
    if (c.kernel == ST_KERNEL_STREAM1D) {
        Geo1 g;
        if (!geo1(p, tb, g)) return fail(ST_ERR_UNSUPPORTED, "1D tiling infeasible");
        Stream1DArgs a;
        std::memset(&a, 0, sizeof(a));
        a.src = src;
        a.dst = dst;
        a.n = p->n[2];
        a.strips = g.strips;
        a.out_w = g.out_w;
        a.halo = g.halo;
        a.tb = tb;
        a.vec_ok = vec_ok && p->n[2] >= 64 * kStream1DVX ? 1 : 0;
        for (int i = 0; i < p->npoints; ++i) a.w[i] = wcan[i];
        e = launch_stream1d(p->dtype, p->radius, p->bc == kPeriodic, a, s);
        if (e != hipSuccess) return hip_fail(e, "stream1d launch");
        return ST_OK;
    }
    if (c.kernel == ST_KERNEL_STREAM2D) {
        Geo2 g;
        if (!geo2(c, p->n[1], p->n[2], tb, g)) return fail(ST_ERR_UNSUPPORTED, "2D tiling infeasible");
        Stream2DArgs a;
        std::memset(&a, 0, sizeof(a));
        a.grids = nullptr;
        a.ngrids = 1;
        a.items = g.items;
        Stream2DGrid& G = a.one;
        G.src = src;
        G.dst = dst;
        G.ny = p->n[1];
        G.nx = p->n[2];
        G.tiles_x = g.tiles_x;
        G.chunks_y = g.chunks_y;
        G.chunk_y = g.chunk_y;
        G.out_w = g.out_w;
        G.hxa = g.hxa;
        G.vec_ok = vec_ok ? 1 : 0;
        G.tb = tb;
        G.tile_begin = 0;
        for (int i = 0; i < p->npoints; ++i) G.w[i] = wcan[i];
        Stream2DKey key = c.k2;
        if (key.tess) {
            // stage 1 (triangles) then stage 2 (inverted triangles at the
            // junctions), in stream order; outflow runs never take this form
            if (fpart) return fail(ST_ERR_UNSUPPORTED, "the tessellated tiling has no outflow twin");
            const int64_t need = tess_bytes(c, g, tb, p->dtype);
            if (!p->tess_buf || need > p->tess_cap)
                return fail(ST_ERR_UNSUPPORTED, "a tessellated pass needs %lld bytes of band scratch, the plan holds %lld",
                            static_cast<long long>(need), static_cast<long long>(p->tess_cap));
            a.tess = p->tess_buf;
            e = launch_stream2d(key, a, s);
            if (e != hipSuccess) return hip_fail(e, "stream2d launch (tessellated stage 1)");
            e = launch_tess2d_band(key, a, s);
            if (e != hipSuccess) return hip_fail(e, "tess2d band launch");
            return ST_OK;
        }
        if (fpart) {
            key.flux = 1;
            if (!stream2d_has(key)) key.tbmax = 8;  // the deepest twin runs any depth
            a.flux_part = fpart;
        }
        e = launch_stream2d(key, a, s);
        if (e != hipSuccess) return hip_fail(e, "stream2d launch");
        return ST_OK;
    }
    if (c.kernel == ST_KERNEL_STREAM3D) {
        Geo3 g;
        if (!geo3(c, p->n, tb, g)) return fail(ST_ERR_UNSUPPORTED, "3D tiling infeasible");
        Stream3DKey key = c.k3;
        key.fast = fast3(p, c, vec_ok) ? 1 : 0;
        key.flux = fpart ? 1 : 0;
        if (key.pipe && (!key.fast || !stream3d_has(key))) {
            // the pipeline has whole-vector rows only (and outflow twins for
            // some tilings): this pass runs on a queued-plane tiling of the
            // plan (same result bit for bit)
            for (const Candidate& o : p->cands)
                if (o.kernel == ST_KERNEL_STREAM3D && !o.k3.pipe && o.k3.tbmax >= tb)
                    return launch_pass(p, o, src, dst, wcan, tb, vec_ok, s, fpart);
            return fail(ST_ERR_UNSUPPORTED, "no queued-plane 3D tiling for a pass of depth %d", tb);
        }
        const int lds = stream3d_lds_bytes(key);
        if (lds > device_lds_limit())
            return fail(ST_ERR_UNSUPPORTED, "tiling needs %d bytes of LDS, the device allows %d", lds,
                        device_lds_limit());
        Stream3DArgs a;
        std::memset(&a, 0, sizeof(a));
        a.src = src;
        a.dst = dst;
        a.nz = p->n[0];
        a.ny = p->n[1];
        a.nx = p->n[2];
        a.tiles_x = g.tiles_x;
        a.tiles_y = g.tiles_y;
        a.chunks_z = g.chunks_z;
        a.out_w = g.out_w;
        a.out_h = g.out_h;
        a.chunk_z = g.chunk_z;
        a.hxa = g.hxa;
        a.hya = g.hya;
        a.vec_ok = vec_ok ? 1 : 0;
        a.tb = tb;
        for (int i = 0; i < p->npoints; ++i) a.w[i] = wcan[i];
        a.flux_part = fpart;
        e = launch_stream3d(key, a, s);
        if (e != hipSuccess) return hip_fail(e, "stream3d launch");
        return ST_OK;
    }
    return fail(ST_ERR_UNSUPPORTED, "kernel family %d unknown", c.kernel);
}

// Outflow runs (zero rule).  A candidate whose 3D kernel has an
// outflow-summing twin keeps its fused depth: every wave sums the outflow of
// its owned cells over the states the pass reads.  Any other candidate runs
// one step per pass, and the band kernel sums the outflow of each state
// before the step reads it.  Either way a one-work-group kernel then adds the
// pass's partial sums to the FP64 accumulator in a fixed order.
bool flux_fused(const st_plan_s* p, const Candidate& c) {
    if (p->bc != kZero) return false;
    if (c.kernel == ST_KERNEL_STREAM2D) {
        if (c.k2.tess) return false;
        Stream2DKey k = c.k2;
        k.flux = 1;
        if (stream2d_has(k)) return true;
        k.tbmax = 8;
        return c.tb <= 8 && stream2d_has(k);
    }
    if (c.kernel != ST_KERNEL_STREAM3D) return false;
    Stream3DKey k = c.k3;
    k.flux = 1;
    k.fast = 1;
    if (!stream3d_has(k)) return false;
    if (c.k3.pipe) return true;  // whole-vector rows only: run_steps checks the grid takes them
    k.fast = 0;
    return stream3d_has(k);
}

// Partial sums one pass of depth tb writes (-1: tiling infeasible).
int64_t flux_parts(const st_plan_s* p, const Candidate& c, bool fused, int tb) {
    if (!fused) return kFluxBandBlocks;
    if (c.kernel == ST_KERNEL_STREAM2D) {
        Geo2 g2;
        if (!geo2(c, p->n[1], p->n[2], tb, g2)) return -1;
        return g2.items;
    }
    Geo3 g;
    if (!geo3(c, p->n, tb, g)) return -1;
    return static_cast<int64_t>(g.tiles_x) * g.tiles_y * g.chunks_z * c.k3.nw;
}

// The partial sums were sized when the plan was made (plan_buffers): a run
// never allocates.
st_status check_flux_parts(const st_plan_s* p, int64_t need) {
    if (!p->flux_part) return fail(ST_ERR_HIP, "the plan holds no outflow buffer (made without a device?)");
    if (need > p->flux_cap)
        return fail(ST_ERR_UNSUPPORTED, "a pass needs %lld outflow partial sums, the plan holds %lld",
                    static_cast<long long>(need), static_cast<long long>(p->flux_cap));
    return ST_OK;
}

// Run `steps` steps with candidate c: grid -> work -> grid ...  With `flux`
// (zero rule only), the outflow of every step is also added to flux[0].
int cand_vx(const st_plan_s* p, const Candidate& c) {
    return c.kernel == ST_KERNEL_STREAM2D   ? c.k2.vx
           : c.kernel == ST_KERNEL_STREAM3D ? c.k3.vx
           : c.kernel == ST_KERNEL_STREAM1D ? kStream1DVX
           : c.kernel == ST_KERNEL_BOX3D    ? box3d_shape(p->dtype, 1).vx
                                            : 1;
}

st_status run_steps(st_plan_s* p, const Candidate& c_sel, void* grid, void* work, const double* wcan,
                    int64_t steps, hipStream_t s, double* flux = nullptr) {
    // The pipeline has whole-vector rows only: on a grid that does not take
    // them (too small, unaligned) the run uses the plan's first other
    // candidate, with its own depth (every candidate gives the same bits; the
    // list always ends with the one-step kernel).
    const Candidate* pick = &c_sel;
    if (c_sel.kernel == ST_KERNEL_STREAM3D && c_sel.k3.pipe) {
        const bool v0 = (p->n[2] % cand_vx(p, c_sel) == 0) && aligned16(grid) && aligned16(work);
        if (!fast3(p, c_sel, v0)) {
            for (const Candidate& o : p->cands)
                if (!(o.kernel == ST_KERNEL_STREAM3D && o.k3.pipe)) {
                    pick = &o;
                    break;
                }
        }
    }
    const Candidate& c_in = *pick;
    const int vx = c_in.kernel == ST_KERNEL_STREAM2D   ? c_in.k2.vx
                   : c_in.kernel == ST_KERNEL_STREAM3D ? c_in.k3.vx
                   : c_in.kernel == ST_KERNEL_STREAM1D ? kStream1DVX
                   : c_in.kernel == ST_KERNEL_BOX3D    ? box3d_shape(p->dtype, 1).vx
                                                       : 1;
    const bool vec_ok = (p->n[2] % vx == 0) && aligned16(grid) && aligned16(work);
    // the pipeline's outflow twin has whole-vector rows only
    const bool fused = flux && flux_fused(p, c_in) &&
                       !(c_in.kernel == ST_KERNEL_STREAM3D && c_in.k3.pipe && !fast3(p, c_in, vec_ok));
    Candidate c = c_in;
    if (flux && !fused) c.tb = 1;
    const int tb = (c.kernel == ST_KERNEL_NAIVE) ? 1 : c.tb;
    bool copy = false;
    const std::vector<int> passes = pass_list(steps, tb, copy);
    const size_t bytes = static_cast<size_t>(plan_cells(p)) * elem_bytes(p->dtype);
    void* src = grid;
    void* dst = work;
    FluxBandArgs fb;
    if (flux) {
        int64_t need = 0;
        for (int t : passes) {
            const int64_t n = flux_parts(p, c, fused, t);
            if (n < 0) return fail(ST_ERR_UNSUPPORTED, "tiling infeasible");
            need = std::max(need, n);
        }
        if (st_status r = check_flux_parts(p, need); r != ST_OK) return r;
        std::memset(&fb, 0, sizeof(fb));
        for (int d = 0; d < 3; ++d) fb.n[d] = p->n[d];
        fb.npoints = p->npoints;
        for (int i = 0; i < p->npoints; ++i) {
            for (int d = 0; d < 3; ++d) {
                fb.off[i][d] = p->off[i][d];
                fb.reach[d] = std::max(fb.reach[d], std::abs(p->off[i][d]));
            }
            fb.w[i] = wcan[i];
        }
    }
    for (int t : passes) {
        if (flux && !fused) {
            fb.src = src;
            if (hipError_t e = launch_flux_band(p->dtype, fb, p->flux_part, kFluxBandBlocks, s); e != hipSuccess)
                return hip_fail(e, "outflow band launch");
        }
        st_status r = launch_pass(p, c, src, dst, wcan, t, vec_ok, s, fused ? p->flux_part : nullptr);
        if (r != ST_OK) return r;
        if (flux) {
            if (hipError_t e = launch_flux_reduce(p->flux_part, flux_parts(p, c, fused, t), flux, s); e != hipSuccess)
                return hip_fail(e, "outflow reduce launch");
        }
        std::swap(src, dst);
    }
    if (copy) ST_HIP(hipMemcpyAsync(grid, work, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync(work->grid)");
    return ST_OK;
}

void describe(const st_plan_s* p, const Candidate& c, int index, st_plan_info* info) {
    std::memset(info, 0, sizeof(*info));
    info->kernel = c.kernel;
    info->tb = c.kernel == ST_KERNEL_NAIVE ? 1 : c.tb;
    info->radius = p->radius;
    info->shape_class = p->cls;
    info->variant = index;
    info->ncandidates = static_cast<int32_t>(p->cands.size());
    if (c.kernel == ST_KERNEL_NAIVE) {
        info->tile_x = info->tile_y = info->tile_z = 1;
        info->block = 256;
        info->workgroups = ceil_div(plan_cells(p), 256);
    } else if (c.kernel == ST_KERNEL_STREAM2D) {
        Geo2 g;
        geo2(c, p->n[1], p->n[2], c.tb, g);
        info->tile_x = g.out_w;
        info->tile_y = g.chunk_y;
        info->tile_z = 1;
        info->block = 256;
        info->workgroups = ceil_div(g.items, 4);
        info->tessellated = c.k2.tess;
    } else if (c.kernel == ST_KERNEL_BOX3D) {
        GeoB g;
        geob(p, c, c.tb, g);
        if (c.bpipe > 0) {
            const BoxPipeShape sh = boxpipe3d_shape(p->dtype, c.bpipe - 1);
            info->tile_x = sh.out_w;
            info->tile_y = sh.out_h;
            info->block = sh.block;
            info->lds_bytes = 2 * (2 * sh.block / 64 + 2) * sh.w * (p->dtype == kF64 ? 8 : 4);
            info->pipeline = c.bpipe;
        } else {
            const Box3DShape sh = box3d_shape(p->dtype, c.tb);
            info->tile_x = sh.out_w;
            info->tile_y = sh.h;
            info->block = sh.block;
        }
        info->tile_z = g.chunk_z;
        info->workgroups = static_cast<int64_t>(g.tiles_x) * g.tiles_y * g.chunks_z;
    } else if (c.kernel == ST_KERNEL_STREAM1D) {
        Geo1 g;
        geo1(p, c.tb, g);
        info->tile_x = g.out_w;
        info->tile_y = info->tile_z = 1;
        info->block = 256;
        info->workgroups = ceil_div(g.strips, 4);
    } else if (c.kernel == ST_KERNEL_VARCOEF3D) {
        info->tile_x = info->tile_y = info->tile_z = 1;
        info->block = 256;
        info->workgroups = ceil_div(plan_cells(p), 256);
    } else if (c.kernel == ST_KERNEL_STREAM3D) {
        Geo3 g;
        geo3(c, p->n, c.tb, g);
        info->tile_x = g.out_w;
        info->tile_y = g.out_h;
        info->tile_z = g.chunk_z;
        info->block = 64 * c.k3.nw;
        info->workgroups = static_cast<int64_t>(g.tiles_x) * g.tiles_y * g.chunks_z;
        info->lds_bytes = stream3d_lds_bytes(c.k3);
        info->pipeline = c.k3.pipe;
    }
}

// ---------------------------------------------------------------------------
// autotune cache: plan key -> chosen candidate, in memory and optionally in a
// text file (one "key<TAB>candidate<TAB>candidates" line per plan)
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;
std::string g_tune_path;

std::string tune_key(const st_plan_s* p) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::string devname = "?";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        devname = std::string(prop.gcnArchName) + ":" + std::to_string(prop.multiProcessorCount);
    std::string k = "v1 " + devname + " nd" + std::to_string(p->ndim) + " t" + std::to_string(p->dtype) + " bc" +
                    std::to_string(p->bc) + (p->batch ? " batch" : " grid");
    if (p->batch) {
        for (const BatchGrid& g : p->grids) k += " " + std::to_string(g.ny) + "x" + std::to_string(g.nx);
    } else {
        k += " " + std::to_string(p->n[0]) + "x" + std::to_string(p->n[1]) + "x" + std::to_string(p->n[2]);
    }
    k += " p";
    for (int i = 0; i < p->npoints; ++i)
        k += " " + std::to_string(p->off[i][0]) + "," + std::to_string(p->off[i][1]) + "," +
             std::to_string(p->off[i][2]);
    return k;
}

bool tune_lookup(st_plan_s* p, const std::string& key) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    const int idx = it->second.first, n = it->second.second;
    if (n != static_cast<int>(p->cands.size()) || idx < 0 || idx >= n) return false;
    p->sel = idx;
    return true;
}

void tune_store(const std::string& key, int idx, int n) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = {idx, n};
    if (g_tune_path.empty()) return;
    // the cache is advisory: a file that cannot be written is left as it is
    FILE* f = std::fopen(g_tune_path.c_str(), "w");
    if (!f) return;
    for (const auto& kv : g_tune) std::fprintf(f, "%s\t%d\t%d\n", kv.first.c_str(), kv.second.first, kv.second.second);
    std::fclose(f);
}

st_status autotune(st_plan_s* p) {
    if (st_status r = need_device(); r != ST_OK) return r;
    if (p->cands.size() <= 1) return ST_OK;
    const std::string tkey = tune_key(p);
    if (tune_lookup(p, tkey)) return ST_OK;
    const size_t bytes = static_cast<size_t>(plan_cells(p)) * elem_bytes(p->dtype);
    void *a = nullptr, *b = nullptr;
    ST_HIP(hipMalloc(&a, bytes), "hipMalloc(autotune)");
    if (hipMalloc(&b, bytes) != hipSuccess) {
        hipFree(a);
        return fail(ST_ERR_NOMEM, "hipMalloc(autotune) failed");
    }
    hipMemset(a, 0, bytes);
    double w[kMaxPoints];
    for (int i = 0; i < p->npoints; ++i) w[i] = (i == 0) ? 1.0 - 0.1 * (p->npoints - 1) / p->npoints : 0.1 / p->npoints;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    double best = 1e300;
    int best_i = p->sel;
    for (size_t i = 0; i < p->cands.size(); ++i) {
        const Candidate& c = p->cands[i];
        const int64_t steps = std::max<int64_t>(8, 4 * c.tb);
        if (run_steps(p, c, a, b, w, steps, nullptr) != ST_OK) continue;  // warm-up
        hipEventRecord(e0, nullptr);
        st_status r = ST_OK;
        for (int rep = 0; rep < 3 && r == ST_OK; ++rep) r = run_steps(p, c, a, b, w, steps, nullptr);
        hipEventRecord(e1, nullptr);
        hipEventSynchronize(e1);
        if (r != ST_OK) continue;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        const double per_step = ms / (3.0 * steps);
        if (per_step < best) { best = per_step; best_i = static_cast<int>(i); }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(a);
    hipFree(b);
    p->sel = best_i;
    tune_store(tkey, best_i, static_cast<int>(p->cands.size()));
    g_last_error.clear();
    return ST_OK;
}

// Key of a run: every argument that ends up inside the launches.
void key_push(std::vector<uint64_t>& k, const void* p) { k.push_back(reinterpret_cast<uintptr_t>(p)); }
void key_push(std::vector<uint64_t>& k, int64_t v) { k.push_back(static_cast<uint64_t>(v)); }
void key_push(std::vector<uint64_t>& k, double v) {
    uint64_t b;
    std::memcpy(&b, &v, sizeof(b));
    k.push_back(b);
}

// With ST_PLAN_GRAPH the launches of a run are captured once on a plan-owned
// stream, instantiated, and replayed with hipGraphLaunch on the caller's
// stream while the arguments (key) stay the same.  A caller that is itself
// capturing gets the plain launches recorded into its own graph.
template <typename F>
st_status run_graphed(st_plan_s* p, const std::vector<uint64_t>& key, hipStream_t s, F&& launches) {
    if (!(p->flags & ST_PLAN_GRAPH) || stream_capturing(s)) return launches(s);
    if (p->graph_exec && key == p->graph_key) {
        ST_HIP(hipGraphLaunch(p->graph_exec, s), "hipGraphLaunch");
        return ST_OK;
    }
    if (!p->cap_stream) return fail(ST_ERR_HIP, "the plan holds no capture stream (made without a device?)");
    if (p->graph_exec) {
        hipGraphExecDestroy(p->graph_exec);
        p->graph_exec = nullptr;
        p->graph_key.clear();
    }
    ST_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    const st_status r = launches(p->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (r != ST_OK) {
        if (g) hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    const hipError_t ei = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) {
        p->graph_exec = nullptr;
        return hip_fail(ei, "hipGraphInstantiate");
    }
    p->graph_key = key;
    ST_HIP(hipGraphLaunch(p->graph_exec, s), "hipGraphLaunch");
    return ST_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// extern "C"
// ---------------------------------------------------------------------------
namespace {
// Checks shared by stencil_run and stencil_run_flux; picks the work buffer
// and rounds the weights.  `nothing` is set when there are no steps.
st_status prepare_run(st_plan_s* plan, void* grid, void*& work, const double* coeffs, const int64_t* shape,
                      int64_t steps, st_boundary bc, hipStream_t s, double* wcan, bool& nothing,
                      bool static_work_space = false) {
    nothing = false;
    if (!plan) return fail(ST_ERR_ARG, "plan is NULL");
    if (plan->batch) return fail(ST_ERR_MISMATCH, "batch plan passed to stencil_run");
    if (plan->flags & ST_PLAN_VARCOEF)
        return fail(ST_ERR_MISMATCH, "variable-coefficient plan passed to stencil_run (use stencil_run_ckpt)");
    if (!shape) return fail(ST_ERR_ARG, "shape is NULL");
    for (int d = 0; d < plan->ndim; ++d)
        if (shape[d] != plan->shape[d])
            return fail(ST_ERR_MISMATCH, "shape[%d] = %lld, plan has %lld", d, static_cast<long long>(shape[d]),
                        static_cast<long long>(plan->shape[d]));
    if (bc != plan->bc) return fail(ST_ERR_MISMATCH, "boundary %d, plan has %d", static_cast<int>(bc), plan->bc);
    if (steps < 0) return fail(ST_ERR_ARG, "steps = %lld < 0", static_cast<long long>(steps));
    if (steps == 0) {
        nothing = true;
        return ST_OK;
    }
    if (!grid) return fail(ST_ERR_ARG, "grid is NULL");
    if (!coeffs) return fail(ST_ERR_ARG, "coeffs is NULL");
    for (int i = 0; i < plan->npoints; ++i)
        if (!std::isfinite(coeffs[i])) return fail(ST_ERR_ARG, "coefficient %d is not finite", i);
    if (st_status r = need_device(); r != ST_OK) return r;
    if (static_work_space) {
        size_t cap = 0;
        if (hipError_t e = static_work(&work, &cap); e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    }
    if (!work) {
        if (!plan->owned_work) return fail(ST_ERR_ARG, "work is NULL and the plan owns none (ST_PLAN_OWN_WORK)");
        work = plan->owned_work;
    }
    if (work == grid) return fail(ST_ERR_ARG, "work aliases grid");
    canonical_weights(plan, coeffs, wcan);
    return ST_OK;
}
}  // namespace

extern "C" {

const char* stencil_last_error(void) { return g_last_error.c_str(); }

const char* stencil_version(void) { return "paper_2303_08365_amd stencil 0.1 (gfx950)"; }

}  // extern "C"

namespace {
st_status plan_buffers(st_plan_s* p);

// stencil_plan without the device buffers and the mirror (the mirror plan of
// a constant-weight adjoint is made this way, host memory only).
st_status make_plan(st_plan_s** out, const st_pattern* pattern, const int64_t* shape, st_dtype storage,
                    st_boundary bc, uint32_t flags, bool full) {
    *out = nullptr;
    if (st_status r = check_pattern(pattern); r != ST_OK) return r;
    if (!shape) return fail(ST_ERR_ARG, "shape is NULL");
    for (int d = 0; d < pattern->ndim; ++d)
        if (shape[d] < 1) return fail(ST_ERR_ARG, "shape[%d] = %lld < 1", d, static_cast<long long>(shape[d]));
    st_plan_s* p = new (std::nothrow) st_plan_s();
    if (!p) return fail(ST_ERR_NOMEM, "plan allocation failed");
    if (st_status r = fill_plan(p, pattern, storage, bc, flags); r != ST_OK) {
        delete p;
        return r;
    }
    for (int d = 0; d < p->ndim; ++d) {
        p->shape[d] = shape[d];
        p->n[3 - p->ndim + d] = shape[d];
    }
    build_candidates(p);
    if (full) {
        st_status r = plan_buffers(p);
        if (r == ST_OK && (flags & ST_PLAN_AUTOTUNE)) r = autotune(p);
        if (r == ST_OK && !(flags & ST_PLAN_VARCOEF)) {
            // the adjoint of a constant-weight sweep is the sweep with every
            // offset negated (same boundary): planned now, so the adjoint
            // call allocates nothing
            std::vector<int32_t> off(static_cast<size_t>(p->npoints) * p->ndim);
            for (int i = 0; i < p->npoints; ++i) {
                const int src = p->perm[i];  // caller's index of canonical point i
                for (int d = 0; d < p->ndim; ++d)
                    off[static_cast<size_t>(src) * p->ndim + d] = -p->off[i][3 - p->ndim + d];
            }
            const st_pattern mp{p->ndim, p->npoints, off.data()};
            r = make_plan(&p->mirror, &mp, p->shape, storage, bc, flags & ST_PLAN_NAIVE, false);
        }
        if (r != ST_OK) {
            stencil_plan_destroy(p);
            return r;
        }
    }
    *out = p;
    return ST_OK;
}
}  // namespace

extern "C" {

st_status stencil_plan(st_plan* out, const st_pattern* pattern, const int64_t* shape, st_dtype storage,
                       st_boundary bc, uint32_t flags) {
    if (!out) return fail(ST_ERR_ARG, "out is NULL");
    st_plan_s* p = nullptr;
    const st_status r = make_plan(&p, pattern, shape, storage, bc, flags, true);
    *out = p;
    return r;
}

st_status stencil_plan_destroy(st_plan plan) {
    if (!plan) return ST_OK;
    if (plan->owned_work) hipFree(plan->owned_work);
    if (plan->flux_part) hipFree(plan->flux_part);
    if (plan->tess_buf) hipFree(plan->tess_buf);
    if (plan->table_dev) hipFree(plan->table_dev);
    if (plan->mirror) stencil_plan_destroy(plan->mirror);
    if (plan->graph_exec) hipGraphExecDestroy(plan->graph_exec);
    if (plan->cap_stream) hipStreamDestroy(plan->cap_stream);
    delete plan;
    return ST_OK;
}

st_status stencil_plan_info(st_plan plan, st_plan_info* info) {
    if (!plan || !info) return fail(ST_ERR_ARG, "plan or info is NULL");
    describe(plan, plan->cands[plan->sel], plan->sel, info);
    return ST_OK;
}

st_status stencil_plan_candidate(st_plan plan, int32_t index, st_plan_info* info) {
    if (!plan || !info) return fail(ST_ERR_ARG, "plan or info is NULL");
    if (index < 0 || index >= static_cast<int32_t>(plan->cands.size()))
        return fail(ST_ERR_ARG, "candidate %d not in 0..%zu", index, plan->cands.size() - 1);
    describe(plan, plan->cands[index], index, info);
    return ST_OK;
}

st_status stencil_plan_select(st_plan plan, int32_t kernel, int32_t tb, int32_t variant) {
    if (!plan) return fail(ST_ERR_ARG, "plan is NULL");
    const int n = static_cast<int>(plan->cands.size());
    if (variant >= 0) {
        if (variant >= n) return fail(ST_ERR_UNSUPPORTED, "candidate %d not in 0..%d", variant, n - 1);
        const Candidate& c = plan->cands[variant];
        if ((kernel >= 0 && c.kernel != kernel) || (tb > 0 && c.tb != tb))
            return fail(ST_ERR_UNSUPPORTED, "candidate %d is kernel %d depth %d", variant, c.kernel, c.tb);
        plan->sel = variant;
        return ST_OK;
    }
    for (int i = 0; i < n; ++i) {
        const Candidate& c = plan->cands[i];
        if ((kernel < 0 || c.kernel == kernel) && (tb <= 0 || c.tb == tb)) {
            plan->sel = i;
            return ST_OK;
        }
    }
    return fail(ST_ERR_UNSUPPORTED, "no candidate with kernel %d and depth %d", kernel, tb);
}

st_status stencil_run(st_plan plan, void* grid, void* work, const double* coeffs, const int64_t* shape,
                      int64_t steps, st_boundary bc, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    double wcan[kMaxPoints];
    bool nothing = false;
    if (st_status r = prepare_run(plan, grid, work, coeffs, shape, steps, bc, s, wcan, nothing); r != ST_OK || nothing)
        return r;
    std::vector<uint64_t> key;
    if (plan->flags & ST_PLAN_GRAPH) {
        key_push(key, grid);
        key_push(key, work);
        key_push(key, steps);
        key_push(key, static_cast<int64_t>(plan->sel));
        for (int i = 0; i < plan->npoints; ++i) key_push(key, wcan[i]);
    }
    const Candidate cand = plan->cands[plan->sel];
    return run_graphed(plan, key, s, [&](hipStream_t st) { return run_steps(plan, cand, grid, work, wcan, steps, st); });
}

st_status stencil_run_noalloc(st_plan plan, void* grid, const double* coeffs, const int64_t* shape, int64_t steps,
                              st_boundary bc, void* stream) {
    if (!plan) return fail(ST_ERR_ARG, "plan is NULL");
    const size_t bytes = static_cast<size_t>(plan_cells(plan)) * elem_bytes(plan->dtype);
    if (!plan->batch && bytes > kStaticWorkBytes)
        return fail(ST_ERR_ARG, "the grid holds %zu bytes; the static work space of stencil_run_noalloc holds %zu",
                    bytes, kStaticWorkBytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double wcan[kMaxPoints];
    bool nothing = false;
    void* work = nullptr;
    if (st_status r = prepare_run(plan, grid, work, coeffs, shape, steps, bc, s, wcan, nothing, true);
        r != ST_OK || nothing)
        return r;
    // eager launches whatever the plan's flags (no graph is instantiated
    // here); inside a caller's capture they are recorded into its graph
    return run_steps(plan, plan->cands[plan->sel], grid, work, wcan, steps, s);
}

st_status stencil_run_flux(st_plan plan, void* grid, void* work, const double* coeffs, const int64_t* shape,
                           int64_t steps, st_boundary bc, double* flux, void* stream) {
    if (!flux) return fail(ST_ERR_ARG, "flux is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double wcan[kMaxPoints];
    bool nothing = false;
    if (st_status r = prepare_run(plan, grid, work, coeffs, shape, steps, bc, s, wcan, nothing); r != ST_OK || nothing)
        return r;
    // a fused candidate of the same depth with an outflow-summing twin
    // stands in for one without (same states bit for bit: every tiling of a
    // plan gives the same grid)
    Candidate cand = plan->cands[plan->sel];
    if (cand.kernel == ST_KERNEL_STREAM3D && !flux_fused(plan, cand))
        for (const Candidate& c : plan->cands)
            if (c.kernel == cand.kernel && c.tb == cand.tb && flux_fused(plan, c)) {
                cand = c;
                break;
            }
    // a periodic grid has no boundary: nothing leaves
    return run_steps(plan, cand, grid, work, wcan, steps, s, plan->bc == kZero ? flux : nullptr);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------
namespace {
st_status batch_autotune(st_plan_s* p);
}  // namespace

extern "C" st_status stencil_batch_plan(st_plan* out, const st_pattern* pattern, int32_t n,
                                        const int64_t* shapes, st_dtype storage, st_boundary bc,
                                        uint32_t flags) {
    if (!out) return fail(ST_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (st_status r = check_pattern(pattern); r != ST_OK) return r;
    if (n < 1) return fail(ST_ERR_ARG, "batch of %d grids", n);
    if (!shapes) return fail(ST_ERR_ARG, "shapes is NULL");
    if (pattern->ndim != 2) return fail(ST_ERR_UNSUPPORTED, "batched plans take 2D patterns");
    for (int64_t i = 0; i < static_cast<int64_t>(n) * 2; ++i)
        if (shapes[i] < 1) return fail(ST_ERR_ARG, "shapes[%lld] < 1", static_cast<long long>(i));
    st_plan_s* p = new (std::nothrow) st_plan_s();
    if (!p) return fail(ST_ERR_NOMEM, "plan allocation failed");
    if (st_status r = fill_plan(p, pattern, storage, bc, flags & ~ST_PLAN_AUTOTUNE); r != ST_OK) {
        delete p;
        return r;
    }
    if (flags & ST_PLAN_VARCOEF) {
        delete p;
        return fail(ST_ERR_UNSUPPORTED, "batched plans take constant weights");
    }
    if (flags & ST_PLAN_OWN_WORK) {
        delete p;
        return fail(ST_ERR_UNSUPPORTED, "batched plans take the caller's work buffers");
    }
    if (p->radius != 1 || (p->cls != kStar && p->cls != kBox)) {
        delete p;
        return fail(ST_ERR_UNSUPPORTED, "batched plans take radius-1 star or box patterns");
    }
    p->batch = true;
    p->flags = flags;
    int64_t maxy = 1, maxx = 1;
    for (int g = 0; g < n; ++g) {
        p->grids.push_back(BatchGrid{shapes[2 * g], shapes[2 * g + 1]});
        maxy = std::max(maxy, shapes[2 * g]);
        maxx = std::max(maxx, shapes[2 * g + 1]);
    }
    p->shape[0] = maxy;
    p->shape[1] = maxx;
    p->n[1] = maxy;
    p->n[2] = maxx;
    build_candidates(p);
    // batch runs need a fused family; drop the naive fallback when one exists
    if (p->cands.size() > 1) p->cands.pop_back();
    st_status r = plan_buffers(p);
    if (r == ST_OK && (flags & ST_PLAN_AUTOTUNE)) r = batch_autotune(p);
    if (r != ST_OK) {
        stencil_plan_destroy(p);
        return r;
    }
    *out = p;
    return ST_OK;
}



namespace {

// Common y-chunk length for the grids of one batched pass: maximises the
// busy fraction of the dispatch rounds over all grids' work items times the
// useful fraction of the streamed rows.
int64_t batch_chunk(const st_plan_s* p, const Candidate& c, int tb, const std::vector<int>& active) {
    const int64_t cap = wave_capacity2(c);
    const int64_t halo = 2 * static_cast<int64_t>(c.k2.radius) * tb;
    int64_t maxny = 1;
    for (int g : active) maxny = std::max(maxny, p->grids[g].ny);
    double best = -1.0;
    int64_t best_len = maxny;
    for (double lf = std::max<int64_t>(8, halo); lf <= static_cast<double>(maxny) * 1.0001; lf *= 1.08) {
        const int64_t len = static_cast<int64_t>(lf);
        int64_t items = 0, rows = 0, streamed = 0;
        for (int g : active) {
            Geo2 geo;
            if (!geo2(c, p->grids[g].ny, p->grids[g].nx, tb, geo, len)) return 0;
            items += geo.items;
            rows += geo.tiles_x * p->grids[g].ny;
            streamed += geo.tiles_x * (p->grids[g].ny + static_cast<int64_t>(geo.chunks_y) * halo);
        }
        const double score =
            std::pow(round_fill(items, cap), 0.25) * static_cast<double>(rows) / static_cast<double>(streamed);
        if (score > best + 1e-9) {
            best = score;
            best_len = len;
        }
    }
    return best_len;
}

}  // namespace

namespace {

// Chunk length of a batch candidate: fixed for the plan (all grids, the
// candidate's depth), so the device table's geometry never depends on the
// run's arguments.
int64_t batch_chunk_of(const st_plan_s* plan, const Candidate& c) {
    if (c.chunk > 0) return c.chunk;
    std::vector<int> all(plan->grids.size());
    for (size_t g = 0; g < all.size(); ++g) all[g] = static_cast<int>(g);
    return batch_chunk(plan, c, c.tb, all);
}

// Work items of every grid of a batch candidate, summed (the launch size of
// every pass; -1 when a grid cannot be tiled).
int64_t batch_items(const st_plan_s* plan, const Candidate& c) {
    const int64_t len = batch_chunk_of(plan, c);
    if (len <= 0) return -1;
    int64_t items = 0;
    for (const BatchGrid& bg : plan->grids) {
        Geo2 geo;
        if (!geo2(c, bg.ny, bg.nx, c.tb, geo, len)) return -1;
        items += geo.items;
    }
    return items;
}

// Build the per-grid descriptor table of a batch run.  Every pass is one
// launch over all grids with the geometry of the candidate's depth; grid g
// runs pass_list(steps[g]) -- `full` passes of that depth, then up to three
// shorter tail passes (a tile with the full depth's halo computes any
// smaller depth exactly) -- and its work-groups return at once in passes
// beyond its own.  Odd passes read the work buffer and write the grid.
st_status batch_table(st_plan_s* plan, const Candidate& c, int32_t n, void* const* grids, void* const* works,
                      const double* coeffs, const int64_t* steps, std::vector<Stream2DGrid>& table, int& npass,
                      int64_t& items, std::vector<int>& copies) {
    const int64_t len = batch_chunk_of(plan, c);
    if (len <= 0) return fail(ST_ERR_UNSUPPORTED, "2D tiling infeasible for the batch");
    table.assign(static_cast<size_t>(n), Stream2DGrid{});
    copies.clear();
    npass = 0;
    items = 0;
    for (int g = 0; g < n; ++g) {
        bool copy = false;
        const std::vector<int> v = pass_list(steps[g], c.tb, copy);
        if (copy) copies.push_back(g);
        int full = 0;
        while (full < static_cast<int>(v.size()) && v[full] == c.tb) ++full;
        if (static_cast<int>(v.size()) - full > 3)
            return fail(ST_ERR_UNSUPPORTED, "pass schedule of grid %d has %zu tail passes", g, v.size() - full);
        npass = std::max(npass, static_cast<int>(v.size()));
        Geo2 geo;
        if (!geo2(c, plan->grids[g].ny, plan->grids[g].nx, c.tb, geo, len))
            return fail(ST_ERR_UNSUPPORTED, "2D tiling infeasible for grid %d", g);
        Stream2DGrid& G = table[g];
        std::memset(&G, 0, sizeof(G));
        G.src = grids[g];
        G.dst = works[g];
        G.ny = plan->grids[g].ny;
        G.nx = plan->grids[g].nx;
        G.tiles_x = geo.tiles_x;
        G.chunks_y = geo.chunks_y;
        G.chunk_y = geo.chunk_y;
        G.out_w = geo.out_w;
        G.hxa = geo.hxa;
        G.vec_ok = (G.nx % c.k2.vx == 0) && aligned16(grids[g]) && aligned16(works[g]);
        G.tb = c.tb;
        G.full = full;
        for (int j = 0; j < 3; ++j) G.tail[j] = full + j < static_cast<int>(v.size()) ? v[full + j] : 0;
        G.tile_begin = items;
        G.items = geo.items;
        G.gid = g;
        canonical_weights(plan, coeffs + static_cast<int64_t>(g) * plan->npoints, G.w);
        items += geo.items;
    }
    return ST_OK;
}

// Put `table` into the plan's device table, in stream order (kernel-argument
// upload: nothing is allocated and nothing waits).  Skipped when the device
// already holds these bytes and nobody else can have rewritten them.
st_status batch_upload(st_plan_s* plan, const std::vector<Stream2DGrid>& table, bool force, hipStream_t s) {
    const size_t bytes = table.size() * sizeof(Stream2DGrid);
    const unsigned char* b = reinterpret_cast<const unsigned char*>(table.data());
    if (!force && !plan->table_foreign && plan->table_shadow.size() == bytes &&
        std::memcmp(plan->table_shadow.data(), b, bytes) == 0)
        return ST_OK;
    if (!plan->table_dev) return fail(ST_ERR_HIP, "the batch plan holds no device table (made without a device?)");
    if (hipError_t e = launch_table_write(plan->table_dev, b, bytes, s); e != hipSuccess)
        return hip_fail(e, "descriptor table upload");
    plan->table_shadow.assign(b, b + bytes);
    return ST_OK;
}

// The passes of a batch run.  With `flux` (one device double per grid),
// every pass runs the outflow-summing twin and a per-grid reduction of its
// partial sums.
st_status batch_launches(const st_plan_s* plan, const Candidate& c, int npass, int64_t items,
                         const std::vector<int>& copies, void* const* grids, void* const* works, hipStream_t s,
                         double* flux = nullptr) {
    const Stream2DGrid* dev = static_cast<const Stream2DGrid*>(plan->table_dev);
    const int n = static_cast<int>(plan->grids.size());
    Stream2DKey key = c.k2;
    if (flux) {
        key.flux = 1;
        if (!stream2d_has(key)) key.tbmax = 8;
    }
    for (int pi = 0; pi < npass; ++pi) {
        Stream2DArgs a;
        std::memset(&a, 0, sizeof(a));
        a.grids = dev;
        a.ngrids = n;
        a.pass = pi;
        a.items = items;
        a.flux_part = flux ? plan->flux_part : nullptr;
        const hipError_t e = launch_stream2d(key, a, s);
        if (e != hipSuccess) return hip_fail(e, "stream2d batch launch");
        if (flux) {
            const hipError_t r = launch_flux_reduce_batch(dev, n, plan->flux_part, flux, s);
            if (r != hipSuccess) return hip_fail(r, "outflow batch reduce launch");
        }
    }
    for (int g : copies) {
        const size_t bytes = static_cast<size_t>(plan->grids[g].ny * plan->grids[g].nx) * elem_bytes(plan->dtype);
        ST_HIP(hipMemcpyAsync(grids[g], works[g], bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync(batch copy)");
    }
    return ST_OK;
}

st_status batch_run_impl(st_plan_s* plan, int32_t n, void* const* grids, void* const* works, const double* coeffs,
                         const int64_t* steps, hipStream_t s, double* flux = nullptr) {
    const Candidate c = plan->cands[plan->sel];
    if (flux && plan->bc != kZero) flux = nullptr;  // a periodic grid has no boundary
    if (c.kernel == ST_KERNEL_NAIVE || (flux && !flux_fused(plan, c))) {
        // pattern without a fused family, or outflow without a summing twin:
        // grid by grid
        st_plan_s one;
        one.ndim = plan->ndim;
        one.dtype = plan->dtype;
        one.bc = plan->bc;
        one.npoints = plan->npoints;
        std::memcpy(one.off, plan->off, sizeof(one.off));
        std::memcpy(one.perm, plan->perm, sizeof(one.perm));
        // the outflow partial sums live in the batch plan's buffer
        one.flux_part = plan->flux_part;
        one.flux_cap = plan->flux_cap;
        st_status r = ST_OK;
        for (int g = 0; g < n && r == ST_OK; ++g) {
            if (steps[g] == 0) continue;
            one.n[1] = plan->grids[g].ny;
            one.n[2] = plan->grids[g].nx;
            double w[kMaxPoints];
            canonical_weights(plan, coeffs + static_cast<int64_t>(g) * plan->npoints, w);
            r = run_steps(&one, c, grids[g], works[g], w, steps[g], s, flux ? flux + g : nullptr);
        }
        one.flux_part = nullptr;
        return r;
    }
    std::vector<Stream2DGrid> table;
    int npass = 0;
    int64_t items = 0;
    std::vector<int> copies;
    if (st_status r = batch_table(plan, c, n, grids, works, coeffs, steps, table, npass, items, copies); r != ST_OK)
        return r;
    if (flux) {
        // eager launches (no graph): the passes with their per-grid reductions
        if (st_status r = check_flux_parts(plan, items); r != ST_OK) return r;
        const bool capturing = stream_capturing(s);
        if (st_status r = batch_upload(plan, table, capturing, s); r != ST_OK) return r;
        // a caller's graph may replay its own table at any later time
        if (capturing) plan->table_foreign = true;
        return batch_launches(plan, c, npass, items, copies, grids, works, s, flux);
    }
    std::vector<uint64_t> key;
    key_push(key, static_cast<int64_t>(plan->sel));
    for (int g = 0; g < n; ++g) {
        key_push(key, grids[g]);
        key_push(key, works[g]);
        key_push(key, steps[g]);
        for (int i = 0; i < plan->npoints; ++i) key_push(key, coeffs[static_cast<int64_t>(g) * plan->npoints + i]);
    }
    if ((plan->flags & ST_PLAN_GRAPH) && !stream_capturing(s)) {
        // the captured graph writes its own table before its passes, so
        // every replay runs with the right descriptors
        const st_status r = run_graphed(plan, key, s, [&](hipStream_t st) {
            if (st_status u = batch_upload(plan, table, true, st); u != ST_OK) return u;
            return batch_launches(plan, c, npass, items, copies, grids, works, st);
        });
        // captured now or replayed: the graph wrote this table (equal keys
        // give equal tables)
        if (r == ST_OK) {
            const unsigned char* b = reinterpret_cast<const unsigned char*>(table.data());
            plan->table_shadow.assign(b, b + table.size() * sizeof(Stream2DGrid));
        } else {
            plan->table_shadow.clear();
        }
        return r;
    }
    const bool capturing = stream_capturing(s);
    if (st_status r = batch_upload(plan, table, capturing, s); r != ST_OK) return r;
    if (capturing) plan->table_foreign = true;
    return batch_launches(plan, c, npass, items, copies, grids, works, s);
}

}  // namespace

namespace {

// Outflow partial sums a plan must hold: the most any pass of any candidate
// writes (the fused twins write one per wave or work item, the band kernel
// kFluxBandBlocks); none for periodic and variable-coefficient plans.
int64_t flux_need(const st_plan_s* p) {
    if (p->bc != kZero || (p->flags & ST_PLAN_VARCOEF)) return 0;
    int64_t need = kFluxBandBlocks;
    for (const Candidate& c : p->cands) {
        if (p->batch) {
            if (c.kernel == ST_KERNEL_STREAM2D) need = std::max(need, batch_items(p, c));
            continue;
        }
        if (!flux_fused(p, c)) continue;
        for (int t = 1; t <= c.tb; ++t) need = std::max(need, flux_parts(p, c, true, t));
    }
    return need;
}

// Every device buffer a plan owns, allocated once here so that no run call
// allocates or waits: the work buffer (ST_PLAN_OWN_WORK), the outflow partial
// sums, the batch descriptor table and the capture stream (ST_PLAN_GRAPH).
// A plan made on a host without a device gets none of them: it can describe
// its tilings but every run call reports the missing device.
st_status plan_buffers(st_plan_s* p) {
    if (!have_device()) return ST_OK;
    if (p->flags & ST_PLAN_OWN_WORK) {
        const size_t bytes = static_cast<size_t>(plan_cells(p)) * elem_bytes(p->dtype);
        if (hipMalloc(&p->owned_work, bytes) != hipSuccess) {
            p->owned_work = nullptr;
            return fail(ST_ERR_NOMEM, "hipMalloc(%zu) for the plan's work buffer failed", bytes);
        }
    }
    const int64_t need = flux_need(p);
    if (need > 0) {
        if (hipMalloc(&p->flux_part, static_cast<size_t>(need) * sizeof(double)) != hipSuccess) {
            p->flux_part = nullptr;
            return fail(ST_ERR_NOMEM, "hipMalloc of %lld outflow partial sums failed", static_cast<long long>(need));
        }
        p->flux_cap = need;
    }
    int64_t tess = 0;
    for (const Candidate& c : p->cands) {
        if (c.kernel != ST_KERNEL_STREAM2D || !c.k2.tess) continue;
        for (int t = 1; t <= c.tb; ++t) {
            Geo2 g;
            if (geo2(c, p->n[1], p->n[2], t, g)) tess = std::max(tess, tess_bytes(c, g, t, p->dtype));
        }
    }
    if (tess > 0) {
        if (hipMalloc(&p->tess_buf, static_cast<size_t>(tess)) != hipSuccess) {
            p->tess_buf = nullptr;
            return fail(ST_ERR_NOMEM, "hipMalloc(%lld) for the tessellated band scratch failed",
                        static_cast<long long>(tess));
        }
        p->tess_cap = tess;
    }
    if (p->batch) {
        const size_t bytes = p->grids.size() * sizeof(Stream2DGrid);
        if (hipMalloc(&p->table_dev, bytes) != hipSuccess) {
            p->table_dev = nullptr;
            return fail(ST_ERR_NOMEM, "hipMalloc(%zu) for the batch descriptor table failed", bytes);
        }
    }
    if (p->flags & ST_PLAN_GRAPH)
        ST_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "hipStreamCreate(capture)");
    return ST_OK;
}

st_status batch_entry(st_plan plan, int32_t n, void* const* grids, void* const* works, const double* coeffs,
                      const int64_t* steps, void* stream, double* flux) {
    if (!plan) return fail(ST_ERR_ARG, "plan is NULL");
    if (!plan->batch) return fail(ST_ERR_MISMATCH, "single-grid plan passed to stencil_batch_run");
    if (n != static_cast<int32_t>(plan->grids.size()))
        return fail(ST_ERR_MISMATCH, "batch of %d grids, plan has %zu", n, plan->grids.size());
    if (!grids || !works || !coeffs || !steps) return fail(ST_ERR_ARG, "NULL batch array");
    int64_t maxsteps = 0;
    for (int g = 0; g < n; ++g) {
        if (steps[g] < 0) return fail(ST_ERR_ARG, "steps[%d] < 0", g);
        if (steps[g] > 0 && (!grids[g] || !works[g])) return fail(ST_ERR_ARG, "grid %d has a NULL buffer", g);
        if (steps[g] > 0 && grids[g] == works[g]) return fail(ST_ERR_ARG, "grid %d: work aliases grid", g);
        maxsteps = std::max(maxsteps, steps[g]);
        for (int i = 0; i < plan->npoints; ++i)
            if (!std::isfinite(coeffs[static_cast<int64_t>(g) * plan->npoints + i]))
                return fail(ST_ERR_ARG, "coefficient %d of grid %d is not finite", i, g);
    }
    if (maxsteps == 0) return ST_OK;
    if (st_status r = need_device(); r != ST_OK) return r;
    return batch_run_impl(plan, n, grids, works, coeffs, steps, static_cast<hipStream_t>(stream), flux);
}
}  // namespace

extern "C" st_status stencil_batch_run(st_plan plan, int32_t n, void* const* grids, void* const* works,
                                       const double* coeffs, const int64_t* steps, void* stream) {
    return batch_entry(plan, n, grids, works, coeffs, steps, stream, nullptr);
}

extern "C" st_status stencil_batch_run_flux(st_plan plan, int32_t n, void* const* grids, void* const* works,
                                            const double* coeffs, const int64_t* steps, double* flux, void* stream) {
    if (!flux) return fail(ST_ERR_ARG, "flux is NULL");
    return batch_entry(plan, n, grids, works, coeffs, steps, stream, flux);
}

namespace {

// ST_PLAN_AUTOTUNE for a batch: time every candidate on scratch grids of the
// batch's shapes and keep the fastest per step.
st_status batch_autotune(st_plan_s* p) {
    if (st_status r = need_device(); r != ST_OK) return r;
    if (p->cands.size() <= 1) return ST_OK;
    const std::string tkey = tune_key(p);
    if (tune_lookup(p, tkey)) return ST_OK;
    const int n = static_cast<int>(p->grids.size());
    std::vector<void*> g(n, nullptr), w(n, nullptr);
    std::vector<double> coeffs(static_cast<size_t>(n) * p->npoints);
    for (int gi = 0; gi < n; ++gi)
        for (int i = 0; i < p->npoints; ++i)
            coeffs[static_cast<size_t>(gi) * p->npoints + i] =
                (i == 0) ? 1.0 - 0.1 * (p->npoints - 1) / p->npoints : 0.1 / p->npoints;
    st_status res = ST_OK;
    for (int gi = 0; gi < n && res == ST_OK; ++gi) {
        const size_t bytes = static_cast<size_t>(p->grids[gi].ny * p->grids[gi].nx) * elem_bytes(p->dtype);
        if (hipMalloc(&g[gi], bytes) != hipSuccess || hipMalloc(&w[gi], bytes) != hipSuccess)
            res = fail(ST_ERR_NOMEM, "hipMalloc(batch autotune) failed");
        else
            hipMemset(g[gi], 0, bytes);
    }
    if (res == ST_OK) {
        const uint32_t flags = p->flags;
        p->flags &= ~ST_PLAN_GRAPH;
        hipEvent_t e0, e1;
        hipEventCreate(&e0);
        hipEventCreate(&e1);
        double best = 1e300;
        int best_i = p->sel;
        for (size_t i = 0; i < p->cands.size(); ++i) {
            p->sel = static_cast<int>(i);
            p->table_shadow.clear();
            const int64_t st = std::max<int64_t>(2, 2 * p->cands[i].tb);
            std::vector<int64_t> steps(n, st);
            if (batch_run_impl(p, n, g.data(), w.data(), coeffs.data(), steps.data(), nullptr) != ST_OK) continue;
            hipEventRecord(e0, nullptr);
            st_status r = batch_run_impl(p, n, g.data(), w.data(), coeffs.data(), steps.data(), nullptr);
            hipEventRecord(e1, nullptr);
            hipEventSynchronize(e1);
            if (r != ST_OK) continue;
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            if (ms / st < best) {
                best = ms / st;
                best_i = static_cast<int>(i);
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        p->sel = best_i;
        p->table_shadow.clear();
        p->flags = flags;
        tune_store(tkey, best_i, static_cast<int>(p->cands.size()));
        g_last_error.clear();
    }
    hipDeviceSynchronize();
    for (int gi = 0; gi < n; ++gi) {
        if (g[gi]) hipFree(g[gi]);
        if (w[gi]) hipFree(w[gi]);
    }
    return res;
}

}  // namespace

// ---------------------------------------------------------------------------
// variable-coefficient forward with checkpoints, and the adjoint
// ---------------------------------------------------------------------------
namespace {

char* at(void* base, int64_t index, size_t bytes) {
    return static_cast<char*>(base) + static_cast<size_t>(index) * bytes;
}

// The z-streaming kernels need tiles that fit inside the grid, whole vector
// rows and planes below 2 GiB; ST_PLAN_NAIVE keeps the one-thread-per-cell
// kernels (the reference form).
bool varcoef_streamable(const st_plan_s* p, bool adjoint, const void* const* ptrs, int nptr) {
    if (p->flags & ST_PLAN_NAIVE) return false;
    int w = 0, h = 0, block = 0;
    varcoef_stream_shape(p->dtype, adjoint, w, h, block);
    const int vx = w / 64;
    if (p->n[2] < w || p->n[1] < h || p->n[2] % vx != 0) return false;
    if (p->n[1] * p->n[2] * elem_bytes(p->dtype) >= (int64_t(1) << 31) || p->n[0] >= (int64_t(1) << 30)) return false;
    for (int i = 0; i < nptr; ++i)
        if (ptrs[i] && !aligned16(ptrs[i])) return false;
    return true;
}

st_status varcoef_launch(const st_plan_s* p, bool adjoint, const void* u, const void* k, const void* lam,
                         void* out, void* grad, double alpha, hipStream_t s) {
    const void* ptrs[5] = {u, k, lam, out, grad};
    if (varcoef_streamable(p, adjoint, ptrs, 5)) {
        VarcoefArgs a;
        std::memset(&a, 0, sizeof(a));
        a.u = u;
        a.k = k;
        a.lam = lam;
        a.out = out;
        a.grad = grad;
        a.nz = p->n[0];
        a.ny = p->n[1];
        a.nx = p->n[2];
        a.alpha = alpha;
        int w = 0, h = 0, block = 0;
        varcoef_stream_shape(p->dtype, adjoint, w, h, block);
        a.tiles_x = static_cast<int32_t>(ceil_div(p->n[2], w));
        a.tiles_y = static_cast<int32_t>(ceil_div(p->n[1], h));
        const int64_t per_plane = static_cast<int64_t>(a.tiles_x) * a.tiles_y;
        const int occ = have_device() ? varcoef_stream_occupancy(p->dtype, adjoint) : 0;
        const int64_t cap = static_cast<int64_t>(device_cus()) * (occ > 0 ? occ : 2);
        const int64_t chunk = std::min<int64_t>(p->n[0], pick_chunk(p->n[0], per_plane, cap, 2, 8));
        a.chunk_z = static_cast<int32_t>(chunk);
        a.chunks_z = static_cast<int32_t>(ceil_div(p->n[0], chunk));
        if (per_plane * a.chunks_z >= (int64_t(1) << 31)) return fail(ST_ERR_UNSUPPORTED, "too many work-groups");
        const hipError_t e = launch_varcoef_stream(p->dtype, adjoint, a, s);
        if (e != hipSuccess) return hip_fail(e, adjoint ? "varcoef adjoint launch" : "varcoef step launch");
        return ST_OK;
    }
    VarcoefArgs a;
    std::memset(&a, 0, sizeof(a));
    a.u = u;
    a.k = k;
    a.lam = lam;
    a.out = out;
    a.grad = grad;
    a.nz = p->n[0];
    a.ny = p->n[1];
    a.nx = p->n[2];
    a.alpha = alpha;
    const hipError_t e = launch_varcoef(p->dtype, adjoint, a, s);
    if (e != hipSuccess) return hip_fail(e, adjoint ? "varcoef adjoint launch" : "varcoef step launch");
    return ST_OK;
}

}  // namespace

extern "C" st_status stencil_run_ckpt(st_plan plan, void* grid, void* work, const void* k, double alpha,
                                      int64_t steps, int64_t every, void* const* ckpts, void* stream) {
    if (!plan) return fail(ST_ERR_ARG, "plan is NULL");
    if (!(plan->flags & ST_PLAN_VARCOEF)) return fail(ST_ERR_MISMATCH, "plan was not made with ST_PLAN_VARCOEF");
    if (steps < 0) return fail(ST_ERR_ARG, "steps = %lld < 0", static_cast<long long>(steps));
    if (ckpts && every < 1) return fail(ST_ERR_ARG, "checkpoint interval %lld < 1", static_cast<long long>(every));
    if (!std::isfinite(alpha)) return fail(ST_ERR_ARG, "alpha is not finite");
    if (steps == 0) return ST_OK;
    if (!grid || !work || !k) return fail(ST_ERR_ARG, "grid, work and k are required");
    if (grid == work) return fail(ST_ERR_ARG, "work aliases grid");
    if (ckpts) {
        for (int64_t c = 0; c < ceil_div(steps, every); ++c)
            if (!ckpts[c]) return fail(ST_ERR_ARG, "checkpoint buffer %lld is NULL", static_cast<long long>(c));
    }
    if (st_status r = need_device(); r != ST_OK) return r;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = static_cast<size_t>(plan_cells(plan)) * elem_bytes(plan->dtype);
    void* cur = grid;
    void* nxt = work;
    for (int64_t t = 0; t < steps; ++t) {
        if (ckpts && t % every == 0)
            ST_HIP(hipMemcpyAsync(ckpts[t / every], cur, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync(checkpoint)");
        if (st_status r = varcoef_launch(plan, false, cur, k, nullptr, nxt, nullptr, alpha, s); r != ST_OK) return r;
        std::swap(cur, nxt);
    }
    if (cur != grid) ST_HIP(hipMemcpyAsync(grid, cur, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync(work->grid)");
    return ST_OK;
}

extern "C" st_status stencil_adjoint_run(st_plan plan, const void* k, double alpha, const double* coeffs,
                                         void* const* ckpts, int64_t every, int64_t steps, void* lambda,
                                         void* grad_k, void* seg, void* work, void* stream) {
    if (!plan) return fail(ST_ERR_ARG, "plan is NULL");
    if (plan->batch) return fail(ST_ERR_MISMATCH, "batch plan passed to stencil_adjoint_run");
    if (steps < 0) return fail(ST_ERR_ARG, "steps = %lld < 0", static_cast<long long>(steps));
    if (steps == 0) return ST_OK;
    if (!lambda || !work) return fail(ST_ERR_ARG, "lambda and work are required");
    if (lambda == work) return fail(ST_ERR_ARG, "work aliases lambda");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = static_cast<size_t>(plan_cells(plan)) * elem_bytes(plan->dtype);
    if (!(plan->flags & ST_PLAN_VARCOEF)) {
        // constant weights: the transpose of u -> sum_p w_p u(x + o_p) is the
        // same sweep with every offset negated
        if (k || grad_k) return fail(ST_ERR_MISMATCH, "k / grad_k given to a constant-weight plan");
        if (!coeffs) return fail(ST_ERR_ARG, "coeffs is NULL");
        if (!plan->mirror) return fail(ST_ERR_MISMATCH, "the plan has no transposed sweep");
        return stencil_run(plan->mirror, lambda, work, coeffs, plan->shape, steps,
                           static_cast<st_boundary>(plan->bc), stream);
    }
    if (!k) return fail(ST_ERR_ARG, "k is required for a variable-coefficient adjoint");
    if (!ckpts || every < 1) return fail(ST_ERR_ARG, "checkpoints and an interval >= 1 are required");
    if (!std::isfinite(alpha)) return fail(ST_ERR_ARG, "alpha is not finite");
    const int64_t nck = ceil_div(steps, every);
    for (int64_t c = 0; c < nck; ++c)
        if (!ckpts[c]) return fail(ST_ERR_ARG, "checkpoint buffer %lld is NULL", static_cast<long long>(c));
    if (std::min(every, steps) > 1 && !seg) return fail(ST_ERR_ARG, "a segment buffer of every-1 states is required");
    if (st_status r = need_device(); r != ST_OK) return r;
    void* cur = lambda;
    void* nxt = work;
    for (int64_t c = nck - 1; c >= 0; --c) {
        const int64_t n0 = c * every;
        const int64_t len = std::min(every, steps - n0);
        // recompute u^{n0+1} .. u^{n0+len-1} into seg[0 .. len-2]
        for (int64_t j = 1; j < len; ++j) {
            const void* prev = (j == 1) ? ckpts[c] : at(seg, j - 2, bytes);
            if (st_status r = varcoef_launch(plan, false, prev, k, nullptr, at(seg, j - 1, bytes), nullptr, alpha, s);
                r != ST_OK)
                return r;
        }
        for (int64_t j = len - 1; j >= 0; --j) {
            const void* u = (j == 0) ? ckpts[c] : at(seg, j - 1, bytes);
            if (st_status r = varcoef_launch(plan, true, u, k, cur, nxt, grad_k, alpha, s); r != ST_OK) return r;
            std::swap(cur, nxt);
        }
    }
    if (cur != lambda) ST_HIP(hipMemcpyAsync(lambda, cur, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync(work->lambda)");
    return ST_OK;
}

// ---------------------------------------------------------------------------
// bandwidth reference
// ---------------------------------------------------------------------------
extern "C" st_status stencil_autotune_cache(const char* path) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (!path) {
        g_tune_path.clear();
        return ST_OK;
    }
    if (!*path) return fail(ST_ERR_ARG, "empty autotune cache path");
    std::map<std::string, std::pair<int, int>> loaded;
    if (FILE* f = std::fopen(path, "r")) {
        char line[8192];
        int lineno = 0;
        while (std::fgets(line, sizeof(line), f)) {
            ++lineno;
            std::string l(line);
            while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
            if (l.empty()) continue;
            const size_t t2 = l.rfind('\t');
            const size_t t1 = t2 == std::string::npos || t2 == 0 ? std::string::npos : l.rfind('\t', t2 - 1);
            char* e1 = nullptr;
            char* e2 = nullptr;
            long idx = 0, n = 0;
            if (t1 != std::string::npos) {
                idx = std::strtol(l.c_str() + t1 + 1, &e1, 10);
                n = std::strtol(l.c_str() + t2 + 1, &e2, 10);
            }
            if (t1 == std::string::npos || e1 != l.c_str() + t2 || *e2 != '\0' || idx < 0 || n < 1 || idx >= n) {
                std::fclose(f);
                return fail(ST_ERR_ARG, "%s:%d: not a 'key<TAB>candidate<TAB>candidates' line", path, lineno);
            }
            loaded[l.substr(0, t1)] = {static_cast<int>(idx), static_cast<int>(n)};
        }
        std::fclose(f);
    }
    for (const auto& kv : loaded) g_tune[kv.first] = kv.second;
    g_tune_path = path;
    return ST_OK;
}

extern "C" st_status stencil_copy(void* dst, const void* src, int64_t bytes, void* stream) {
    if (bytes < 0) return fail(ST_ERR_ARG, "bytes = %lld < 0", static_cast<long long>(bytes));
    if (bytes == 0) return ST_OK;
    if (!dst || !src) return fail(ST_ERR_ARG, "dst and src are required");
    if (!aligned16(dst) || !aligned16(src)) return fail(ST_ERR_ARG, "dst and src must be 16-byte aligned");
    const uintptr_t d = reinterpret_cast<uintptr_t>(dst), s0 = reinterpret_cast<uintptr_t>(src);
    if (d < s0 + static_cast<uintptr_t>(bytes) && s0 < d + static_cast<uintptr_t>(bytes))
        return fail(ST_ERR_ARG, "dst and src overlap");
    if (st_status r = need_device(); r != ST_OK) return r;
    const hipError_t e = launch_copy(dst, src, bytes, device_cus(), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return ST_OK;
}
