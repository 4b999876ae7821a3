// pipe3d_impl.h -- 3D radius-1 stars (7 points) with T_b steps fused per
// pass: the z pipeline kept as partial sums, one LDS exchange per plane.
//
// Same tiling as the 2.5-D kernel of stream3d_impl.h (paper Sec. 4.1: an xy
// tile held on chip while the work-group streams along z; Sec. 4.2: tiles
// staged on chip so global accesses stay coalesced): lane L of wave w holds
// columns X0 + L*VX .. +VX-1 of rows Y0 + w*K .. +K-1, x neighbours come
// from the lane's own registers or lane +-1 through DPP, y neighbours from
// the wave's own rows or, for its first and last row, from the neighbouring
// waves through LDS.  What differs is how the z direction is kept.
//
// The canonical order of a 7-point star evaluates the point at z+1 last:
//   u'(z) = fma(w6, u(z+1), P(z)),
//   P(z)  = w0 u(z) -> z-1 -> y-1 -> x-1 -> x+1 -> y+1  (one mul, five fma).
// Level l (the state after l fused steps) therefore keeps only two planes
// per lane: its previous plane u_l(z-1) and the partial sum P_l(z-1) of the
// next level.  When plane u_l(z) arrives, fma(w6, u_l(z), P_l(z-1)) is
// already the finished plane u_{l+1}(z-1) -- it needs no neighbour exchange
// -- so one iteration first runs that completion through all levels (phase
// A: level 0's new input plane yields level 1's plane, which yields level
// 2's, ...; the last level's is stored), and right behind each completion
// starts the level's next partial sum with its two terms that need no
// neighbour, w0 u_l(z) and w1 u_l(z-1); u_l(z) then replaces u_l(z-1), so a
// level holds two planes at every point of the iteration.  Then the edge
// rows of every level's new plane go through LDS behind ONE barrier (phase
// B), and the partial sums take their y and x terms (phase C).  Against
// three queued planes per level and a barrier per level this needs about
// two thirds of the registers and a quarter of the barriers (four fused
// steps), with the same arithmetic bit for bit.
//
// Input planes arrive one of two ways.  PD planes ahead in registers: the
// loads of plane z+PD are issued when plane z enters.  Or (LQ) two planes
// ahead through a two-slot LDS queue that buffer-to-LDS loads fill: no
// register holds a plane in flight, the loads have two iterations to land,
// and a wave reads its rows back from LDS when the plane enters.  Counted on
// MI355X, the loads' latency is what a pass with one plane ahead in
// registers waits for.
//
// Level l is exact on the register tile shrunk by l columns per side in x
// (the DPP shifts bring 0 into lanes 0 and 63) and, in y, by l-1 rows per
// side (level 0's rows just outside the tile are loaded once per tile and
// pass through LDS like the wave edge rows, later levels see 0 there).  The
// planner's tiles keep hxa >= tb columns and hya >= tb-1 rows of halo.  Under
// the zero rule a tile that would cross the grid edge is moved inward to
// touch it, where those zeros are the ghost layer, so edge tiles are exact up
// to the edge.  A plane outside the grid is a ghost plane: level 0 loads it
// as 0 (empty descriptor range); a deeper level's value there is never used,
// because the z weights that would read it are set to 0 for that iteration
// (scalar selects, nothing per element; exact for finite states).
//
// Memory access: one buffer descriptor per plane (range = the plane, empty
// for a ghost plane) and, per row, one 32-bit vector offset fixed for the
// whole pass (the row and the lane's columns), so a load or store of a whole
// row is one instruction with no per-row descriptor.  Rows that are not
// output rows, lanes whose columns lie outside the output tile, and halo rows
// outside the grid use an offset past the range's end: the hardware drops
// such a store and returns 0 for such a load.  (The range check covers the
// vector offset only, so the scalar offset stays 0.)  Needs planes below
// 2 GiB, whole-vector rows, and under the zero rule nx >= 64*VX, ny >= NW*K.
#pragma once

#include <utility>

#include "dev_common.h"
#include "registry.h"

namespace st {

namespace p3d {

template <typename TS, int TBMAX, int VX, int K, int NW, bool PER, int NB, int PD, bool FLX, bool LQ>
struct Pipe {
    using S = Storage<TS>;
    using TC = typename S::TC;
    static_assert(NW >= 2 && K >= 2, "a tile needs two waves of two rows");
    static_assert(NB == 1 || NB == 2, "one or two LDS buffers");
    static_assert(PD >= 1 && PD <= 2, "one or two planes prefetched");
    static_assert(!FLX || !PER, "outflow: zero rule only (a periodic grid has no boundary)");
    static constexpr int W = 64 * VX;
    static constexpr int H = NW * K;
    using TC0 = typename Storage<TS>::TC;
    // Partial sums started in phase A (early form: two planes a level) or in
    // phase C (late form: three).  Measured on MI355X at four fused steps:
    // late is faster for 4 x 2 FP64 values a lane (1075 against 1035
    // Gcell/s, 512^3), early for 8 x 2 FP32 values (1623 against 1557);
    // wider FP64 tiles and the LDS queue need early's registers.
    static constexpr bool kEarly = LQ || sizeof(TC0) < 8 || K * VX > 8;
    // LQ: the input planes come through a two-slot LDS queue filled by
    // buffer-to-LDS loads two iterations ahead (no registers held by the
    // prefetch); one dwordx4 per lane and row, four rows per wave
    static_assert(!LQ || (VX * sizeof(TS) == 16 && K == 4 && NB == 1 && PD == 2),
                  "LDS queue: 16-byte rows, four rows per wave, one exchange buffer, two planes ahead");
    // LDS rows of one level: slot 0 the tile's halo row above, 2w+1 and 2w+2
    // the first and last row of wave w, 2*NW+1 the halo row below, 2*NW+2 a
    // sink for waves that own no halo row.  Wave w reads its row above from
    // slot 2w and its row below from slot 2w+3.
    static constexpr int SLOTS = 2 * NW + 3;
    static constexpr int LEVEL_ELEMS = SLOTS * W;
    static constexpr int BUF_ELEMS = TBMAX * LEVEL_ELEMS;
    static constexpr int DYN_BYTES = NB * BUF_ELEMS * static_cast<int>(sizeof(TC));
    // queue slot: row 0 the halo row above, 1..H the tile's rows, H+1 the
    // halo row below, H+2 a sink for the waves that own no halo row
    static constexpr int QROWS = H + 3;
    static constexpr int QROW_BYTES = W * static_cast<int>(sizeof(TS));
    static constexpr int QSLOT_BYTES = QROWS * QROW_BYTES;
    static constexpr int Q_BYTES = LQ ? 2 * QSLOT_BYTES : 16;
    static constexpr int LDS_BYTES = DYN_BYTES + (LQ ? Q_BYTES : 0);
    static constexpr uint32_t kOut = 0x80000000u;  // past the end of any plane (planes < 2 GiB)
    static constexpr int32_t kRsrcWord3 = 0x00020000;  // gfx9: raw 32-bit data
    static constexpr int kNT = 2;                      // stores: non-temporal

    struct Ctx {
        const TS* src;
        TS* dst;
        int32_t nz;
        uint32_t plane_bytes, row_bytes;
        int32_t zs, ze, zlast;
        uint32_t lo[K];        // byte offset of this lane's columns in each of the wave's rows
        uint32_t so[K];        // same for the stores; kOut outside the output tile
        uint32_t ho;           // same for this wave's halo row; kOut: none, or a ghost row
        int hslot;             // the halo row's LDS slot
        int lane, wave;
        // LQ: LDS byte address of this lane's 16 bytes of its first row in
        // queue slot 0, and the queue row its halo load lands in
        uint32_t qaddr, qhaddr;
        TS* qbase;             // the queue (slot 0, row 0)
        int qhrow;
        TC w[7];
        // FLX: the outflow of the owned cells of every state a step reads
        double* fpart;         // this wave's partial sum
        int32_t ny, nx, xl, yw, ox0, ox1, oy0, oy1;
        bool fx;               // the output tile reaches the x faces
        TC lx;                 // weight leaving through this lane's face column (0: none)
        uint32_t rowmask;      // bit k: the wave's row k lies inside the output tile (wave-uniform)
        bool fzy;              // the z chunk reaches a z face, or the wave owns a y-face row
        int32_t k0, k1;        // the wave's rows that the tile owns: k0 <= k < k1
    };

    static __device__ __forceinline__ bool zghost(int32_t z, int32_t nz) {
        return !PER && static_cast<uint32_t>(z) >= static_cast<uint32_t>(nz);
    }
    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_in(const Ctx& c, int32_t zin) {
        const int32_t zz = PER ? wrap_idx(zin < c.zlast ? zin : c.zlast, c.nz) : (zin < c.zlast ? zin : c.zlast);
        const bool out = zghost(zz, c.nz);
        const TS* base = out ? c.src : c.src + static_cast<int64_t>(zz) * (c.plane_bytes / sizeof(TS));
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<TS*>(base), 0, out ? 0 : c.plane_bytes, kRsrcWord3);
    }
    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_out(const Ctx& c, int32_t z) {
        const bool ok = static_cast<uint32_t>(z - c.zs) < static_cast<uint32_t>(c.ze - c.zs);
        TS* base = ok ? c.dst + static_cast<int64_t>(z) * (c.plane_bytes / sizeof(TS)) : c.dst;
        return __builtin_amdgcn_make_buffer_rsrc(base, 0, ok ? c.plane_bytes : 0, kRsrcWord3);
    }

    static __device__ __forceinline__ void ldrow(__amdgpu_buffer_rsrc_t r, uint32_t vo, TC (&v)[VX]) {
        constexpr int kBytes = VX * static_cast<int>(sizeof(TS));
        static_assert(kBytes == 8 || kBytes % 16 == 0, "rows are read in 8- or 16-byte pieces");
        TS vals[VX];
        if constexpr (kBytes % 16 == 0) {
            u32x4 raw[kBytes / 16];
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i)
                raw[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, vo + 16 * i, 0, 0));
            __builtin_memcpy(vals, raw, kBytes);
        } else {
            const u32x2 raw = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(r, vo, 0, 0));
            __builtin_memcpy(vals, &raw, kBytes);
        }
#pragma unroll
        for (int e = 0; e < VX; ++e) v[e] = S::widen(vals[e]);
    }
    static __device__ __forceinline__ void strow(__amdgpu_buffer_rsrc_t r, uint32_t vo, const TC (&v)[VX]) {
        constexpr int kBytes = VX * static_cast<int>(sizeof(TS));
        TS vals[VX];
#pragma unroll
        for (int e = 0; e < VX; ++e) vals[e] = S::narrow(v[e]);
        if constexpr (kBytes % 16 == 0) {
            u32x4 raw[kBytes / 16];
            __builtin_memcpy(raw, vals, kBytes);
#pragma unroll
            for (int i = 0; i < kBytes / 16; ++i) __builtin_amdgcn_raw_buffer_store_b128(raw[i], r, vo + 16 * i, 0, kNT);
        } else {
            u32x2 raw;
            __builtin_memcpy(&raw, vals, kBytes);
            __builtin_amdgcn_raw_buffer_store_b64(raw, r, vo, 0, kNT);
        }
    }

    // The wave's K rows of input plane zin and its halo row (if it owns one).
    static __device__ __forceinline__ void load_plane(const Ctx& c, int32_t zin, TC (&v)[K][VX], TC (&h)[VX]) {
        const __amdgpu_buffer_rsrc_t r = plane_in(c, zin);
#pragma unroll
        for (int k = 0; k < K; ++k) ldrow(r, c.lo[k], v[k]);
        ldrow(r, c.ho, h);
    }

    // Workgroup barrier.  LQ: LDS writes drained and the barrier, without
    // the release fence of __syncthreads, which would also wait for the
    // queue's loads in flight.  LDS is the only memory the waves exchange.
    static __device__ __forceinline__ void sync() {
        if constexpr (LQ) {
            __asm__ volatile("" ::: "memory");
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt: any
            __builtin_amdgcn_s_barrier();
            __asm__ volatile("" ::: "memory");
        } else {
            __syncthreads();
        }
    }
    static __device__ __forceinline__ uint32_t lds_addr(const void* p) {
        return static_cast<uint32_t>(
            reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) const void*)(p)));
    }
    // LQ: plane zin's rows of this wave (and its halo row) into queue slot q,
    // straight from HBM to LDS; lanes out of a range (ghost plane, ghost
    // halo row, no halo row) land as 0.  K + 1 loads per wave.
    static __device__ __forceinline__ void q_issue(const Ctx& c, int q, int32_t zin) {
        const __amdgpu_buffer_rsrc_t r = plane_in(c, zin);
        unsigned char* slot = reinterpret_cast<unsigned char*>(c.qbase) + q * QSLOT_BYTES;
#pragma unroll
        for (int k = 0; k < K; ++k)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                r, (__attribute__((address_space(3))) void*)(slot + (1 + c.wave * K + k) * QROW_BYTES), 16, c.lo[k],
                0, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            r, (__attribute__((address_space(3))) void*)(slot + c.qhrow * QROW_BYTES), 16, c.ho, 0, 0, 0);
    }
    // LQ: this lane's share of queue slot q: its K rows and its halo row.
    // The loads that filled the slot were issued two iterations ago; every
    // iteration issues K + 1 queue loads and K stores, so once at most 2K + 1
    // memory operations are outstanding (the previous iteration's), they are
    // done.  The compiler sees neither these reads nor this wait, so it adds
    // no wait of its own for the queue's loads.
    static __device__ __forceinline__ void q_read(const Ctx& c, int q, TC (&v)[K][VX], TC (&h)[VX]) {
        const uint32_t a = c.qaddr + q * QSLOT_BYTES;
        const uint32_t ah = c.qhaddr + q * QSLOT_BYTES;
        u32x4 r0, r1, r2, r3, rh;
        __asm__ volatile(
            "s_waitcnt vmcnt(9)\n\t"
            "ds_read_b128 %0, %5\n\t"
            "ds_read_b128 %1, %5 offset:%7\n\t"
            "ds_read_b128 %2, %5 offset:%8\n\t"
            "ds_read_b128 %3, %5 offset:%9\n\t"
            "ds_read_b128 %4, %6\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(rh)
            : "v"(a), "v"(ah), "n"(QROW_BYTES), "n"(2 * QROW_BYTES), "n"(3 * QROW_BYTES)
            : "memory");
        const u32x4 rr[K + 1] = {r0, r1, r2, r3, rh};
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            TS vals[VX];
            __builtin_memcpy(vals, &rr[k], 16);
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                if (k < K) v[k < K ? k : 0][e] = S::widen(vals[e]);
                else h[e] = S::widen(vals[e]);
            }
        }
    }

    // Outflow (FLX, zero rule, reading of the absorbing ghost layer): a step
    // moves w_p u(c) from c to c - off_p; what would land outside the grid
    // has left.  For the 7-point star a face cell loses, per face it lies on,
    // the weight of the point that looks across that face: z = 0 -> w6,
    // z = nz-1 -> w1, y = 0 -> w5, y = ny-1 -> w2, x = 0 -> w4, x = nx-1 -> w3.
    // z and y parts: FP64 per cell, behind wave-uniform branches (nonzero
    // only on the first / last plane and on the rows of the waves that own a
    // y-face row).  x part: edge tiles touch the x faces, so a face column is
    // column 0 of lane 0 or column VX-1 of lane 63; per iteration a lane adds
    // up its face column over the rows of every state (T_b * K values,
    // compute precision, a 0 factor for rows and planes the tile does not own,
    // so every wave does the same work between two barriers) and adds the sum,
    // times the face's leaving weight, to its FP64 total.  (One wave doing
    // more, as when unowned rows took a slower path, holds back all eight:
    // FP32 1250 against 1343 Gcell/s with outflow at 512^3.)
    static __device__ __forceinline__ double leave_z(const Ctx& c, int32_t z) {
        return (z + 1 >= c.nz ? static_cast<double>(c.w[1]) : 0.0) + (z < 1 ? static_cast<double>(c.w[6]) : 0.0);
    }
    static __device__ __forceinline__ double leave_y(const Ctx& c, int32_t y) {
        return (y + 1 >= c.ny ? static_cast<double>(c.w[2]) : 0.0) + (y < 1 ? static_cast<double>(c.w[5]) : 0.0);
    }
    static __device__ __forceinline__ double leave_x(const Ctx& c, int32_t x) {
        return (x + 1 >= c.nx ? static_cast<double>(c.w[3]) : 0.0) + (x < 1 ? static_cast<double>(c.w[4]) : 0.0);
    }
    static __device__ __forceinline__ bool own_x(const Ctx& c, int32_t x) {
        return static_cast<uint32_t>(x - c.ox0) < static_cast<uint32_t>(c.ox1 - c.ox0);
    }
    struct Flux {
        double fl;     // the outflow so far
    };
    // z and y parts of one plane of one state
    static __device__ __forceinline__ void flux_zy(const Ctx& c, Flux& f, int32_t z, const TC (&v)[K][VX]) {
        if (static_cast<uint32_t>(z - c.zs) >= static_cast<uint32_t>(c.ze - c.zs)) return;
        const bool zb = z < 1 || z + 1 >= c.nz;
        const double cz = zb ? leave_z(c, z) : 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int32_t y = c.yw + k;
            if (static_cast<uint32_t>(y - c.oy0) >= static_cast<uint32_t>(c.oy1 - c.oy0)) continue;
            const bool yb = y < 1 || y + 1 >= c.ny;
            if (!zb && !yb) continue;
            const double czy = yb ? cz + leave_y(c, y) : cz;
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                // opaque copy: keeps the conversion inside this rare branch
                // (otherwise it is hoisted into every plane)
                TC u = v[k][e];
                __asm__ volatile("" : "+v"(u));
                f.fl = own_x(c, c.xl + e) ? fma(static_cast<double>(u), czy, f.fl) : f.fl;
            }
        }
    }
    // All states of one iteration (planes zin - l of levels l < TB): the z / y
    // parts per state; the x part as one compute-precision sum of the lane's
    // face column (column 0 of lane 0, column VX-1 of lane 63; c.lx, the
    // weight leaving through that face, is 0 elsewhere) over the owned rows of
    // the states whose plane is owned, weighted into the FP64 total once per
    // iteration.
    template <int TB>
    static __device__ __forceinline__ void flux_add(const Ctx& c, Flux& f, int32_t zin, const TC (&cur)[TB][K][VX]) {
        if (c.fzy) {
#pragma unroll
            for (int l = 0; l < TB; ++l) flux_zy(c, f, zin - l, cur[l]);
        }
        if (c.fx) {
            // every wave the same work (the waves meet at a barrier every
            // plane): rows outside the output tile and planes outside the
            // chunk enter with a 0 factor (exact for finite states)
            const bool hi = c.lane == 63;
            TC col = TC(0);
#pragma unroll
            for (int l = 0; l < TB; ++l) {
                const int32_t z = zin - l;
                TC cl = TC(0);
#pragma unroll
                for (int k = 0; k < K; ++k)
                    cl = fma_c(hi ? cur[l][k][VX - 1] : cur[l][k][0], (c.rowmask >> k & 1u) ? TC(1) : TC(0), cl);
                col += static_cast<uint32_t>(z - c.zs) < static_cast<uint32_t>(c.ze - c.zs) ? cl : TC(0);
            }
            f.fl = fma(static_cast<double>(col), static_cast<double>(c.lx), f.fl);
        }
    }
    static __device__ __forceinline__ void flux_store_sum(const Ctx& c, double t) {
        t = wave_sum(t);
        if (c.lane == 0) *c.fpart = t;
    }
    static __device__ __forceinline__ void flux_store(const Ctx& c, const Flux& f) { flux_store_sum(c, f.fl); }

    template <int TB>
    struct State {
        TC prev[TB][K][VX];   // u_l(z-1)
        TC pend[TB][K][VX];   // P_l(z-1): u_{l+1}(z-1) short of its z+1 term
        TC pf[PD][K][VX];     // prefetched input planes
        TC hpf[PD][VX];       // their halo rows
        Flux fx;              // FLX only
    };

    // One iteration: input plane zin enters level 0.
    template <int TB, int J>
    static __device__ __forceinline__ void step(const Ctx& c, int32_t it, int32_t zfirst, State<TB>& s, TC* lds) {
        const int32_t zin = zfirst + it;
        TC cur[K][VX];  // the new plane of the level at hand: u_l(zin-l)
        TC* buf = lds + (NB == 2 ? (it & 1) * BUF_ELEMS : 0);
        if constexpr (LQ) {
            TC halo[VX];
            q_read(c, it & 1, cur, halo);
            TC* lv = buf + c.hslot * W + c.lane * VX;
#pragma unroll
            for (int e = 0; e < VX; ++e) lv[e] = halo[e];
            q_issue(c, it & 1, zin + 2);  // the slot's reads are done
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int e = 0; e < VX; ++e) cur[k][e] = s.pf[J][k][e];
            // Level 0's halo row goes to LDS before the next plane's loads
            // are issued: its registers are then free to receive them.
            // (Written later, the halo would stay live across the loads, the
            // compiler would load into other registers and copy back at the
            // end of the iteration -- a wait for loads issued in the same
            // iteration.)  The buffer is free: its last readers passed the
            // previous barrier.
            TC* lv = buf + c.hslot * W + c.lane * VX;
#pragma unroll
            for (int e = 0; e < VX; ++e) lv[e] = s.hpf[J][e];
            load_plane(c, zin + PD, s.pf[J], s.hpf[J]);
        }

        // FP64: phases A and B run at a raised wave priority: they form the
        // chain each arriving plane starts, while phase C (back at the base
        // priority) only prepares the next iteration (measured +0.7 %; no
        // gain for FP32, a loss for bfloat16).
        if constexpr (sizeof(TC) == 8) __builtin_amdgcn_s_setprio(1);
        // phase A, level by level: u_{l+1}(zin-l-1) = fma(w6, u_l(zin-l),
        // P_l(zin-l-1)) (a ghost plane zin-l, where levels >= 1 hold junk,
        // enters with weight 0); the last level's plane is stored.  Early
        // form: then the next partial sum of level l takes its first two
        // terms, which need no neighbour, w0 u_l(zin-l) and w1 u_l(zin-l-1),
        // and u_l(zin-l) replaces u_l(zin-l-1), so across the LDS exchange a
        // level keeps two planes.  Late form: every level's new plane is kept
        // (three planes a level) and all of the partial sum waits for phase C,
        // off the chain of completions that each input plane starts.
        TC nw[kEarly ? 1 : TB][K][VX];
#pragma unroll
        for (int l = 0; l < TB; ++l) {
            const TC w6 = (l > 0 && zghost(zin - l, c.nz)) ? TC(0) : c.w[6];
            TC nxt[K][VX];
            if (l + 1 < TB) {
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int e = 0; e < VX; ++e) nxt[k][e] = S::round(fma_c(w6, cur[k][e], s.pend[l][k][e]));
            } else {
                const __amdgpu_buffer_rsrc_t r = plane_out(c, zin - TB);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    TC o[VX];
#pragma unroll
                    for (int e = 0; e < VX; ++e) o[e] = fma_c(w6, cur[k][e], s.pend[l][k][e]);
                    strow(r, c.so[k], o);
                }
            }
            if constexpr (kEarly) {
                const TC w1 = (l > 0 && zghost(zin - l - 1, c.nz)) ? TC(0) : c.w[1];
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int e = 0; e < VX; ++e) {
                        s.pend[l][k][e] = fma_c(w1, s.prev[l][k][e], c.w[0] * cur[k][e]);
                        s.prev[l][k][e] = cur[k][e];
                    }
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int e = 0; e < VX; ++e) nw[kEarly ? 0 : l][k][e] = cur[k][e];
            }
            if (l + 1 < TB) {
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int e = 0; e < VX; ++e) cur[k][e] = nxt[k][e];
            }
        }

        // the states this pass reads, one plane of each: u_l(zin - l)
        if constexpr (FLX) {
            if constexpr (kEarly) flux_add<TB>(c, s.fx, zin, s.prev);
            else flux_add<TB>(c, s.fx, zin, nw);
        }

        // phase B: edge rows of every level's new plane through LDS, one
        // barrier
#pragma unroll
        for (int l = 0; l < TB; ++l) {
            const TC (&u)[K][VX] = kEarly ? s.prev[l] : nw[kEarly ? 0 : l];
            TC* lv = buf + l * LEVEL_ELEMS + c.lane * VX;
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                lv[(2 * c.wave + 1) * W + e] = u[0][e];
                lv[(2 * c.wave + 2) * W + e] = u[K - 1][e];
            }
        }
        sync();
        if constexpr (sizeof(TC) == 8) __builtin_amdgcn_s_setprio(0);

        // phase C: the (rest of the) next partial sums; the neighbour rows of
        // every level are read first, one LDS round trip
        TC above[TB][VX], below[TB][VX];
#pragma unroll
        for (int l = 0; l < TB; ++l) {
            const TC* lv = buf + l * LEVEL_ELEMS + c.lane * VX;
#pragma unroll
            for (int e = 0; e < VX; ++e) {
                above[l][e] = lv[(2 * c.wave) * W + e];
                below[l][e] = lv[(2 * c.wave + 3) * W + e];
            }
        }
#pragma unroll
        for (int l = 0; l < TB; ++l) {
            const TC (&u)[K][VX] = kEarly ? s.prev[l] : nw[kEarly ? 0 : l];
            const TC w1 = (l > 0 && zghost(zin - l - 1, c.nz)) ? TC(0) : c.w[1];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const TC lft = from_lower_z(u[k][VX - 1]);
                const TC rgt = from_upper_z(u[k][0]);
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    TC acc = kEarly ? s.pend[l][k][e] : fma_c(w1, s.prev[l][k][e], c.w[0] * u[k][e]);
                    acc = fma_c(c.w[2], k > 0 ? u[k > 0 ? k - 1 : 0][e] : above[l][e], acc);
                    acc = fma_c(c.w[3], e > 0 ? u[k][e > 0 ? e - 1 : 0] : lft, acc);
                    acc = fma_c(c.w[4], e + 1 < VX ? u[k][e + 1 < VX ? e + 1 : 0] : rgt, acc);
                    acc = fma_c(c.w[5], k + 1 < K ? u[k + 1 < K ? k + 1 : 0][e] : below[l][e], acc);
                    s.pend[l][k][e] = acc;
                    if constexpr (!kEarly) s.prev[l][k][e] = u[k][e];
                }
            }
        }
        if constexpr (NB == 1) sync();  // the next iteration rewrites the buffer
    }

    template <int TB, int... J>
    static __device__ __forceinline__ void group(const Ctx& c, int32_t base, int32_t zfirst, State<TB>& s, TC* lds,
                                                 std::integer_sequence<int, J...>) {
        (step<TB, J>(c, base + J, zfirst, s, lds), ...);
    }
    template <int TB, int... J>
    static __device__ __forceinline__ void tail(const Ctx& c, int32_t base, int32_t nit, int32_t zfirst, State<TB>& s,
                                                TC* lds, std::integer_sequence<int, J...>) {
        ((base + J < nit ? step<TB, J>(c, base + J, zfirst, s, lds) : void()), ...);
    }

    template <int TB>
    static __device__ __forceinline__ void run_tb(Ctx& c, TC* lds) {
        const int32_t zfirst = c.zs - TB;
        const int32_t nit = (c.ze - c.zs) + 2 * TB;
        c.zlast = zfirst + nit - 1;
        // halo slots of the levels >= 1 hold 0 for the whole pass
        for (int i = threadIdx.x; i < NB * TBMAX * W; i += blockDim.x) {
            const int b = i / (TBMAX * W), l = (i / W) % TBMAX, col = i % W;
            if (l == 0) continue;
            TC* lv = lds + b * BUF_ELEMS + l * LEVEL_ELEMS;
            lv[col] = TC(0);
            lv[(2 * NW + 1) * W + col] = TC(0);
        }
        __syncthreads();
        State<TB> s;
        s.fx.fl = 0.0;
#pragma unroll
        for (int l = 0; l < TB; ++l)
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    s.prev[l][k][e] = TC(0);
                    s.pend[l][k][e] = TC(0);
                }
        // stores into an empty range (the hardware drops them): the loop is
        // then entered, as it is repeated, with each plane's loads followed by
        // one plane's stores, which the waits at the top of the loop count
        const __amdgpu_buffer_rsrc_t none = plane_out(c, c.ze);
        TC zero[VX];
#pragma unroll
        for (int e = 0; e < VX; ++e) zero[e] = TC(0);
        if constexpr (LQ) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                q_issue(c, p, zfirst + p);
#pragma unroll
                for (int k = 0; k < K; ++k) strow(none, c.so[k], zero);
            }
            for (int32_t it = 0; it < nit; ++it) step<TB, 0>(c, it, zfirst, s, lds);
            // the last two iterations' queue loads (planes past the chunk,
            // never read) land before the work-group's LDS is released
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt, lgkmcnt: any
        } else {
#pragma unroll
            for (int p = 0; p < PD; ++p) load_plane(c, zfirst + p, s.pf[p], s.hpf[p]);
#pragma unroll
            for (int k = 0; k < K; ++k) strow(none, c.so[k], zero);
            int32_t base = 0;
            for (; base + PD <= nit; base += PD)
                group<TB>(c, base, zfirst, s, lds, std::make_integer_sequence<int, PD>{});
            tail<TB>(c, base, nit, zfirst, s, lds, std::make_integer_sequence<int, PD>{});
        }
        if constexpr (FLX) flux_store(c, s.fx);
    }

    static __device__ __forceinline__ void run(const Stream3DArgs& a, TC* lds, TS* lq) {
        Ctx c;
        c.lane = threadIdx.x & 63;
        c.wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
        const uint32_t tiles = static_cast<uint32_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
        const uint32_t item = static_cast<uint32_t>(xcd_remap(blockIdx.x, gridDim.x));
        if constexpr (FLX) c.fpart = a.flux_part + static_cast<int64_t>(blockIdx.x) * NW + c.wave;
        if (item >= tiles) {
            if constexpr (FLX) flux_store_sum(c, 0.0);
            return;
        }
        const uint32_t txy = item / static_cast<uint32_t>(a.tiles_x);
        const int32_t tx = static_cast<int32_t>(item - txy * a.tiles_x);
        const int32_t ty = static_cast<int32_t>(txy % static_cast<uint32_t>(a.tiles_y));
        const int32_t cz = static_cast<int32_t>(txy / static_cast<uint32_t>(a.tiles_y));
        const int32_t nx = static_cast<int32_t>(a.nx), ny = static_cast<int32_t>(a.ny);
        c.src = static_cast<const TS*>(a.src);
        c.dst = static_cast<TS*>(a.dst);
        c.nz = static_cast<int32_t>(a.nz);
        c.row_bytes = static_cast<uint32_t>(nx) * sizeof(TS);
        c.plane_bytes = static_cast<uint32_t>(ny) * c.row_bytes;
        const int32_t ox0 = tx * a.out_w, oy0 = ty * a.out_h;
        const int32_t ox1 = ox0 + a.out_w < nx ? ox0 + a.out_w : nx;
        const int32_t oy1 = oy0 + a.out_h < ny ? oy0 + a.out_h : ny;
        int32_t X0 = ox0 - a.hxa, Y0 = oy0 - a.hya;
        if (!PER) {  // move edge tiles inward (exact: the ghost layer is 0)
            X0 = X0 < 0 ? 0 : (X0 + W > nx ? nx - W : X0);
            Y0 = Y0 < 0 ? 0 : (Y0 + H > ny ? ny - H : Y0);
        }
        const int32_t xl = X0 + c.lane * VX;
        const int32_t yw = Y0 + c.wave * K;
        const int32_t x0 = PER ? wrap_idx(xl, nx) : xl;
        const bool xown = xl >= ox0 && xl < ox1;  // whole lanes: out_w, hxa and nx are multiples of VX
#pragma unroll
        for (int k = 0; k < K; ++k) {
            // zero rule: rows yw + k lie in the grid (the tile was moved inward)
            const int32_t yk = PER ? wrap_idx(yw + k, ny) : yw + k;
            const uint32_t off = static_cast<uint32_t>(yk * nx + x0) * sizeof(TS);
            c.lo[k] = off;
            c.so[k] = (xown && yw + k >= oy0 && yw + k < oy1) ? off : kOut;
        }
        {
            // halo rows: wave 0 the row above the tile, wave NW-1 the row below
            const bool top = c.wave == 0, bot = c.wave == NW - 1;
            const int32_t hy = top ? Y0 - 1 : Y0 + H;
            const bool valid = (top || bot) && (PER || static_cast<uint32_t>(hy) < static_cast<uint32_t>(ny));
            const int32_t hyw = PER ? wrap_idx(hy, ny) : hy;
            c.ho = valid ? static_cast<uint32_t>(hyw * nx + x0) * sizeof(TS) : kOut;
            c.hslot = top ? 0 : (bot ? 2 * NW + 1 : 2 * NW + 2);
            if constexpr (LQ) {
                c.qbase = lq;
                c.qhrow = top ? 0 : (bot ? H + 1 : H + 2);
                const uint32_t q0 = lds_addr(lq) + static_cast<uint32_t>(c.lane) * 16u;
                c.qaddr = q0 + static_cast<uint32_t>((1 + c.wave * K) * QROW_BYTES);
                c.qhaddr = q0 + static_cast<uint32_t>(c.qhrow * QROW_BYTES);
            }
        }
        c.zs = cz * a.chunk_z;
        c.ze = c.zs + a.chunk_z < c.nz ? c.zs + a.chunk_z : c.nz;
        if constexpr (FLX) {
            c.ny = ny;
            c.nx = nx;
            c.xl = xl;
            c.yw = yw;
            c.ox0 = ox0;
            c.ox1 = ox1;
            c.oy0 = oy0;
            c.oy1 = oy1;
            c.fx = ox0 < 1 || ox1 > nx - 1;
            bool fy = false;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int32_t y = yw + k;
                fy = fy || (y >= oy0 && y < oy1 && (y < 1 || y + 1 >= ny));
            }
            c.k0 = oy0 - yw > 0 ? oy0 - yw : 0;
            c.k1 = oy1 - yw < K ? oy1 - yw : K;
            c.fzy = fy || c.zs < 1 || c.ze > c.nz - 1;
        }
#pragma unroll
        for (int p = 0; p < 7; ++p) c.w[p] = static_cast<TC>(a.w[p]);
        if constexpr (FLX) {
            const int32_t xf = c.xl + (c.lane == 63 ? VX - 1 : 0);
            c.lx = static_cast<TC>(own_x(c, xf) ? leave_x(c, xf) : 0.0);
            uint32_t m = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) m |= (k >= c.k0 && k < c.k1) ? 1u << k : 0u;
            c.rowmask = __builtin_amdgcn_readfirstlane(m);
        }
        const int tb = a.tb;
        if constexpr (TBMAX >= 4) if (tb == 4) return run_tb<4>(c, lds);
        if constexpr (TBMAX >= 3) if (tb == 3) return run_tb<3>(c, lds);
        if constexpr (TBMAX >= 2) if (tb == 2) return run_tb<2>(c, lds);
        run_tb<1>(c, lds);
    }
};

template <typename TS, int TBMAX, int VX, int K, int NW, bool PER, int NB, int PD, bool FLX, bool LQ>
__global__ __launch_bounds__(64 * NW) void pipe3d_kernel(const Stream3DArgs a) {
    using P = Pipe<TS, TBMAX, VX, K, NW, PER, NB, PD, FLX, LQ>;
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (LQ) {
        __shared__ __align__(16) unsigned char lq[P::Q_BYTES];
        P::run(a, reinterpret_cast<typename P::TC*>(smem), reinterpret_cast<TS*>(lq));
    } else {
        P::run(a, reinterpret_cast<typename P::TC*>(smem), nullptr);
    }
}

template <typename TS, int TBMAX, int VX, int K, int NW, bool PER, int NB, int PD, bool FLX, bool LQ>
void launch(const Stream3DArgs& a, hipStream_t s) {
    using P = Pipe<TS, TBMAX, VX, K, NW, PER, NB, PD, FLX, LQ>;
    const int64_t tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z;
    hipLaunchKernelGGL((pipe3d_kernel<TS, TBMAX, VX, K, NW, PER, NB, PD, FLX, LQ>),
                       dim3(static_cast<unsigned>(tiles)), dim3(64 * NW), P::DYN_BYTES, s, a);
}

template <typename TS, int TBMAX, int VX, int K, int NW, bool PER, int NB, int PD, bool FLX, bool LQ>
int occ_of() {
    using P = Pipe<TS, TBMAX, VX, K, NW, PER, NB, PD, FLX, LQ>;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pipe3d_kernel<TS, TBMAX, VX, K, NW, PER, NB, PD, FLX, LQ>,
                                                     64 * NW, P::DYN_BYTES) != hipSuccess)
        n = 0;
    return n;
}

template <typename TS> constexpr int32_t dtype_of();
template <> constexpr int32_t dtype_of<double>() { return kF64; }
template <> constexpr int32_t dtype_of<float>() { return kF32; }
template <> constexpr int32_t dtype_of<bf16s>() { return kBF16; }

// Key: radius 1, whole-vector rows, pipe = NB * 10 + PD, plus 100 for the LDS
// queue (no late / ylds).
#define P3D_ENTRY(TS, TBM, VX, K, NW, PER, NB, PD, FLX, LQ)                                                  \
    Entry3{Stream3DKey{dtype_of<TS>(), (PER) ? kPeriodic : kZero, 1, TBM, VX, K, NW, 1, 0, 0, FLX,            \
                       (NB) * 10 + (PD) + ((LQ) ? 100 : 0)},                                                  \
           &launch<TS, TBM, VX, K, NW, PER, NB, PD, FLX, LQ>,                                                 \
           Pipe<TS, TBM, VX, K, NW, PER, NB, PD, FLX, LQ>::LDS_BYTES, &occ_of<TS, TBM, VX, K, NW, PER, NB, PD, FLX, LQ>}
#define P3D_BC(TS, TBM, VX, K, NW, NB, PD) \
    P3D_ENTRY(TS, TBM, VX, K, NW, false, NB, PD, false, false), P3D_ENTRY(TS, TBM, VX, K, NW, true, NB, PD, false, false)
// the LDS-queue form (one exchange buffer, two planes ahead)
#define P3D_LQ(TS, TBM, VX, NW) \
    P3D_ENTRY(TS, TBM, VX, 4, NW, false, 1, 2, false, true), P3D_ENTRY(TS, TBM, VX, 4, NW, true, 1, 2, false, true)
// outflow-summing twins (zero rule)
#define P3D_FLUX(TS, TBM, VX, K, NW, NB, PD) P3D_ENTRY(TS, TBM, VX, K, NW, false, NB, PD, true, false)
#define P3D_LQ_FLUX(TS, TBM, VX, NW) P3D_ENTRY(TS, TBM, VX, 4, NW, false, 1, 2, true, true)

}  // namespace p3d
}  // namespace st
