// registry.h -- instantiation tables of the templated kernel families.  Each
// instantiation unit (s2d_*.hip, s3d_*.hip) compiles one slice of the
// variants in parallel with the others and exports its table here.
#pragma once

#include "internal.h"

namespace st {

struct Entry2 {
    Stream2DKey key;
    void (*fn)(const Stream2DArgs&, hipStream_t);
    int (*occ)();  // resident work-groups per CU on the current device (0 = unknown)
};
struct Entry3 {
    Stream3DKey key;
    void (*fn)(const Stream3DArgs&, hipStream_t);
    int lds;
    int (*occ)();
};
struct Table2 {
    const Entry2* e;
    int n;
};
struct Table3 {
    const Entry3* e;
    int n;
};

Table2 s2d_table_f64();
Table2 s2d_table_f32();
Table2 s2d_table_bf16();
Table2 s2d_table_r2();
Table2 s2d_table_tess();
Table3 s3d_table_r1_f64();
Table3 s3d_table_r1_f32();
Table3 s3d_table_r1_bf16();
Table3 s3d_table_r4();
Table3 p3d_table_r1();

}  // namespace st
