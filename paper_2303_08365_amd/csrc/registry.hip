// registry.hip -- look up a kernel variant across the instantiation units.
#include "registry.h"

namespace st {

namespace {
const Entry2* find2(const Stream2DKey& k) {
    const Table2 tabs[] = {s2d_table_f64(), s2d_table_f32(), s2d_table_bf16(), s2d_table_r2(), s2d_table_tess()};
    for (const Table2& t : tabs)
        for (int i = 0; i < t.n; ++i) {
            const Stream2DKey& e = t.e[i].key;
            if (e.dtype == k.dtype && e.bc == k.bc && e.cls == k.cls && e.radius == k.radius &&
                e.tbmax == k.tbmax && e.vx == k.vx && e.flux == k.flux && e.tess == k.tess)
                return &t.e[i];
        }
    return nullptr;
}
const Entry3* find3(const Stream3DKey& k) {
    const Table3 tabs[] = {s3d_table_r1_f64(), s3d_table_r1_f32(), s3d_table_r1_bf16(), s3d_table_r4(),
                           p3d_table_r1()};
    for (const Table3& t : tabs)
        for (int i = 0; i < t.n; ++i) {
            const Stream3DKey& e = t.e[i].key;
            if (e.dtype == k.dtype && e.bc == k.bc && e.radius == k.radius && e.tbmax == k.tbmax &&
                e.vx == k.vx && e.k == k.k && e.nw == k.nw && e.fast == k.fast && e.late == k.late &&
                e.ylds == k.ylds && e.flux == k.flux && e.pipe == k.pipe)
                return &t.e[i];
        }
    return nullptr;
}
}  // namespace

bool stream2d_has(const Stream2DKey& k) { return find2(k) != nullptr; }

int stream2d_occupancy(const Stream2DKey& k) {
    const Entry2* e = find2(k);
    return e ? e->occ() : 0;
}

int stream3d_occupancy(const Stream3DKey& k) {
    const Entry3* e = find3(k);
    return e ? e->occ() : 0;
}

hipError_t launch_stream2d(const Stream2DKey& k, const Stream2DArgs& a, hipStream_t s) {
    const Entry2* e = find2(k);
    if (!e) return hipErrorInvalidValue;
    if (a.items <= 0) return hipSuccess;
    e->fn(a, s);
    return hipGetLastError();
}

bool stream3d_has(const Stream3DKey& k) { return find3(k) != nullptr; }

int stream3d_lds_bytes(const Stream3DKey& k) {
    const Entry3* e = find3(k);
    return e ? e->lds : -1;
}

hipError_t launch_stream3d(const Stream3DKey& k, const Stream3DArgs& a, hipStream_t s) {
    const Entry3* e = find3(k);
    if (!e) return hipErrorInvalidValue;
    if (static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.chunks_z <= 0) return hipSuccess;
    e->fn(a, s);
    return hipGetLastError();
}

}  // namespace st
