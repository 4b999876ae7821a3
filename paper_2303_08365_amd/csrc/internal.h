// internal.h -- argument blocks and launchers shared by the host side
// (stencil_abi.cpp) and the kernel translation units.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace st {

constexpr int kMaxPoints = 125;
constexpr int kMaxRadius = 4;

enum Dtype : int32_t { kF64 = 0, kF32 = 1, kBF16 = 2 };
enum Bc : int32_t { kZero = 0, kPeriodic = 1 };
enum Cls : int32_t { kGeneral = 0, kStar = 1, kBox = 2 };

// ----------------------------------------------------------------------------
// one step per launch, any pattern (the reference form of every other kernel)
// ----------------------------------------------------------------------------
struct NaiveArgs {
    const void* src;
    void* dst;
    int64_t n[3];              // nz, ny, nx (leading 1s for lower ndim)
    int32_t npoints;
    int32_t bc;
    int32_t off[kMaxPoints][3];  // canonical order, centre first
    double w[kMaxPoints];        // weights already rounded to compute precision
};
hipError_t launch_naive(int dtype, const NaiveArgs& a, hipStream_t s);

// ----------------------------------------------------------------------------
// 2D: rows streamed through registers, T_b fused steps per pass
// ----------------------------------------------------------------------------
// A wave owns an x strip of 64*VX columns (its register tile) and walks the
// rows of one y chunk.  Level l of the pipeline holds 2R+1 rows of step l.
struct Stream2DGrid {
    const void* src;
    void* dst;
    int64_t ny, nx;
    int32_t tiles_x;     // strips across x
    int32_t chunks_y;    // y chunks
    int32_t chunk_y;     // output rows per chunk
    int32_t out_w;       // output columns per strip = 64*VX - 2*hxa
    int32_t hxa;         // redundant halo columns each side (multiple of VX)
    int32_t vec_ok;      // rows and base are aligned for whole-vector access
    int32_t tb;          // fused steps this pass (<= template depth); batch: the full depth
    int32_t full;        // batch: passes of depth tb, then up to 3 tail passes
    int32_t tail[3];     // batch: depths of the tail passes (0 = no such pass)
    int64_t tile_begin;  // first work item of this grid in the batch
    int64_t items;       // work items of this grid (outflow reduction)
    int32_t gid;         // batch entry the descriptor belongs to (outflow reduction)
    double w[32];        // canonical-order weights
};
struct Stream2DArgs {
    const Stream2DGrid* grids;  // device table (batch) or nullptr
    Stream2DGrid one;           // used when grids == nullptr
    int32_t ngrids;
    int32_t pass;               // batch: pass index (odd passes read dst and write src;
                                // a grid whose schedule has no such pass does nothing)
    int64_t items;              // total (grid, strip, chunk) work items
    double* flux_part;          // outflow variants: one partial sum per work item
    void* tess;                 // tessellated tiling: the band rows of every row junction
};
// Instantiation key for the 2D family.
struct Stream2DKey {
    int32_t dtype, bc, cls, radius, tbmax, vx;
    int32_t flux;  // also sums the outflow of every step of the pass (zero rule, single grid)
    int32_t tess;  // tessellated tiling along y (tess2d.hip): stage 1 of a pass (single grid)
};
hipError_t launch_stream2d(const Stream2DKey& k, const Stream2DArgs& a, hipStream_t s);
// Stage 2 of a tessellated pass (tess2d.hip): the inverted triangles at the
// row junctions, one wave per (junction, strip); `a` as for stage 1.
hipError_t launch_tess2d_band(const Stream2DKey& k, const Stream2DArgs& a, hipStream_t s);
// Band rows per junction (both arrays, per strip) of a tessellated pass.
constexpr int tess_band_rows(int radius, int tb) { return 2 * radius * (tb + 1); }
bool stream2d_has(const Stream2DKey& k);
int stream2d_occupancy(const Stream2DKey& k);  // work-groups per CU, 0 if unknown

// ----------------------------------------------------------------------------
// 3D star: planes streamed along z, K rows per lane, LDS edge-row exchange
// ----------------------------------------------------------------------------
struct Stream3DArgs {
    const void* src;
    void* dst;
    int64_t nz, ny, nx;
    int32_t tiles_x, tiles_y, chunks_z;
    int32_t out_w, out_h, chunk_z;
    int32_t hxa, hya;    // redundant halo columns/rows inside the register tile
    int32_t vec_ok;
    int32_t tb;
    double w[32];        // canonical-order weights (6R+1 used)
    double* flux_part;   // outflow variants: one partial sum per wave (work-group * NW + wave)
};
struct Stream3DKey {
    int32_t dtype, bc, radius, tbmax, vx, k, nw;
    int32_t fast;  // whole-vector rows (see stream3d_impl.h)
    int32_t late;  // one-plane prefetch issued after step 0 (fewer registers)
    int32_t ylds;  // step-0 y neighbours through LDS too, the tile's halo rows loaded once
    int32_t flux;  // also sums the outflow of every step of the pass (zero rule)
    int32_t pipe;  // 0: queued planes (stream3d_impl.h); NB*10+PD: radius-1 partial-sum
                   // pipeline with NB LDS buffers and PD prefetched planes (pipe3d_impl.h)
};
hipError_t launch_stream3d(const Stream3DKey& k, const Stream3DArgs& a, hipStream_t s);
bool stream3d_has(const Stream3DKey& k);
int stream3d_lds_bytes(const Stream3DKey& k);
int stream3d_occupancy(const Stream3DKey& k);  // work-groups per CU, 0 if unknown

// ----------------------------------------------------------------------------
// 1D stars: a wave holds a strip of 64*VX cells and takes T_b steps in VGPRs
// ----------------------------------------------------------------------------
constexpr int kStream1DVX = 16;
struct Stream1DArgs {
    const void* src;
    void* dst;
    int64_t n;
    int64_t strips;      // strips of out_w owned cells
    int32_t out_w;       // owned cells per strip = 64*VX - 2*halo
    int32_t halo;        // stale cells at each end of a strip (>= R*tb, multiple of VX)
    int32_t tb;          // steps this pass
    int32_t vec_ok;      // whole-vector access (n % VX == 0, n >= 64*VX, 16-byte aligned)
    double w[9];         // canonical-order weights (2R+1 used)
};
bool stream1d_has(int dtype, int radius);
hipError_t launch_stream1d(int dtype, int radius, bool periodic, const Stream1DArgs& a, hipStream_t s);

// ----------------------------------------------------------------------------
// 3D radius-1 boxes (27 points): one step per pass, planes streamed along z
// ----------------------------------------------------------------------------
struct Box3DArgs {
    const void* src;
    void* dst;
    int64_t nz, ny, nx;
    int32_t tiles_x, tiles_y, chunks_z, chunk_z;
    int32_t tb;          // steps per pass: 1 or 2
    double w[27];        // canonical-order weights
};
struct Box3DShape {
    int vx;              // columns per lane
    int w;               // register tile width 64*vx
    int h;               // owned rows per tile (rows per wave x waves)
    int out_w;           // owned columns per tile
    int block;           // threads per work-group
};
Box3DShape box3d_shape(int dtype, int tb);
hipError_t launch_box3d(int dtype, bool periodic, bool fast, const Box3DArgs& a, hipStream_t s);
// two fused steps, partial sums along z, one LDS row exchange per plane
// (zero rule, whole-vector rows; Box3DArgs.tb = 2)
struct BoxPipeShape {
    int vx, k;           // columns and rows per lane
    int w, h;            // register tile: 64*vx columns x k*waves rows
    int out_w, out_h;    // owned columns and rows per tile
    int block;           // threads per work-group
};
int boxpipe3d_variants(int dtype);
BoxPipeShape boxpipe3d_shape(int dtype, int variant);
hipError_t launch_boxpipe3d(int dtype, int variant, const Box3DArgs& a, hipStream_t s);

// ----------------------------------------------------------------------------
// variable-coefficient 3D heat step (zero rule) and its adjoint
// ----------------------------------------------------------------------------
struct VarcoefArgs {
    const void* u;      // state the step reads (u^n)
    const void* k;      // conductivity
    const void* lam;    // adjoint only: dL/du^{n+1}
    void* out;          // u^{n+1} (forward) or dL/du^n (adjoint)
    void* grad;         // adjoint only: dL/dk accumulator (+=), may be null
    int64_t nz, ny, nx;
    double alpha;
    // filled by launch_varcoef: work-group index -> (row, x block), row -> (z, y)
    uint32_t nxb, nxb_m, nxb_l, ny_m, ny_l;
    // streaming kernels: tiles of varcoef_stream_shape(), chunks of planes
    int32_t tiles_x, tiles_y, chunks_z, chunk_z;
};
hipError_t launch_varcoef(int dtype, bool adjoint, const VarcoefArgs& a, hipStream_t s);
// z-streaming step / adjoint (needs nx >= w, ny >= h, planes below 2 GiB)
void varcoef_stream_shape(int dtype, bool adjoint, int& w, int& h, int& block);
hipError_t launch_varcoef_stream(int dtype, bool adjoint, const VarcoefArgs& a, hipStream_t s);
int varcoef_stream_occupancy(int dtype, bool adjoint);  // work-groups per CU, 0 if unknown

// ----------------------------------------------------------------------------
// outflow across the zero-rule boundary (FP64 partial sums + fixed-order reduce)
// ----------------------------------------------------------------------------
struct FluxBandArgs {
    const void* src;           // the state a step reads
    int64_t n[3];
    int32_t npoints;
    int32_t reach[3];          // largest |offset| along z, y, x
    int32_t off[kMaxPoints][3];
    double w[kMaxPoints];      // weights already rounded to compute precision
};
constexpr int kFluxBandBlocks = 512;
// one partial per work-group into part[0 .. nblocks)
hipError_t launch_flux_band(int dtype, const FluxBandArgs& a, double* part, int nblocks, hipStream_t s);
// flux[0] += sum of part[0 .. n) (one work-group, fixed order)
hipError_t launch_flux_reduce(const double* part, int64_t n, double* flux, hipStream_t s);
// batch: for each of the `count` descriptors of a pass, flux[gid] += sum of
// part[tile_begin .. tile_begin + items) (one work-group per descriptor)
hipError_t launch_flux_reduce_batch(const struct Stream2DGrid* table, int count, const double* part, double* flux,
                                    hipStream_t s);

// plain streaming copy (bandwidth reference); 16-byte aligned buffers
hipError_t launch_copy(void* dst, const void* src, int64_t bytes, int cus, hipStream_t s);
// writes `bytes` host bytes to device memory `dst` in stream order: the bytes
// travel as kernel arguments (captured with the launch), so the host buffer
// may be reused at once and nothing waits; dst 4-byte aligned, bytes % 4 == 0
hipError_t launch_table_write(void* dst, const void* src, size_t bytes, hipStream_t s);

// Static work space (noalloc.hip): a file-scope device array of
// kStaticWorkBytes, its address on the current device looked up once per
// device.  Used only by stencil_run_noalloc.
constexpr size_t kStaticWorkBytes = size_t(64) << 20;
hipError_t static_work(void** ptr, size_t* bytes);

}  // namespace st
