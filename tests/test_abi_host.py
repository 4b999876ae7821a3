"""Host-side checks of libstencil.so: it loads, exports every declared symbol,
classifies patterns, plans tilings, and rejects bad arguments before any
launch.  No kernel runs here."""
import ctypes
import os
import re
import struct
import subprocess
import tempfile

import pytest

import paper_2303_08365_amd as st
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x100000  # never dereferenced: every case below fails host-side checks


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names.update(re.findall(r"\b(stencil_\w+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = st.library()
    names = _declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert b"gfx950" in lib.stencil_version()


def test_star_and_box_classification_and_families():
    p = st.Plan(synth.star_offsets(3, 1), (64, 64, 64), "f64")
    i = p.info()
    assert i["kernel"] == st.KERNEL_STREAM3D and i["shape_class"] == 1 and i["radius"] == 1
    p = st.Plan(synth.star_offsets(3, 4), (64, 64, 64), "f32", "periodic")
    assert p.info()["radius"] == 4 and p.info()["kernel"] == st.KERNEL_STREAM3D
    p = st.Plan(synth.box_offsets(2, 1), (100, 300), "f32")
    assert p.info()["shape_class"] == 2 and p.info()["kernel"] == st.KERNEL_STREAM2D
    p = st.Plan(synth.star_offsets(2, 1), (100, 300), "bf16")
    assert p.info()["kernel"] == st.KERNEL_STREAM2D
    # general point sets and radius-2 3D boxes run on the one-step kernel
    p = st.Plan([(0, 0), (0, 1), (-2, 0)], (50, 50), "f64")
    assert p.info()["shape_class"] == 0 and p.info()["kernel"] == st.KERNEL_NAIVE
    p = st.Plan(synth.box_offsets(3, 1), (20, 20, 20), "f64")
    assert p.info()["shape_class"] == 2 and p.info()["kernel"] == st.KERNEL_BOX3D
    p = st.Plan(synth.box_offsets(3, 2), (20, 20, 20), "f64")
    assert p.info()["shape_class"] == 2 and p.info()["kernel"] == st.KERNEL_NAIVE
    # 1D stars of radius 1 and 2 run on the strip kernel; other 1D sets one step at a time
    p = st.Plan(synth.star_offsets(1, 2), (1000,), "f64")
    assert p.info()["kernel"] == st.KERNEL_STREAM1D
    p = st.Plan(synth.star_offsets(1, 3), (1000,), "f64")
    assert p.info()["kernel"] == st.KERNEL_NAIVE
    p = st.Plan([(0,), (2,)], (1000,), "f64")
    assert p.info()["kernel"] == st.KERNEL_NAIVE
    p = st.Plan(synth.star_offsets(3, 1), (64, 64, 64), "f64", naive=True)
    assert p.info()["kernel"] == st.KERNEL_NAIVE and p.info()["ncandidates"] == 1


def test_candidates_and_select():
    p = st.Plan(synth.star_offsets(3, 1), (512, 512, 512), "f64")
    cands = p.candidates()
    assert len(cands) >= 3 and cands[-1]["kernel"] == st.KERNEL_NAIVE
    for c in cands:
        assert c["workgroups"] > 0 and c["tile_x"] > 0
    tb2 = [k for k, c in enumerate(cands) if c["tb"] == 2]
    assert tb2
    p.select(variant=tb2[0])
    assert p.info()["tb"] == 2 and p.info()["variant"] == tb2[0]
    p.select(kernel=st.KERNEL_NAIVE)
    assert p.info()["kernel"] == st.KERNEL_NAIVE
    with pytest.raises(st.StencilError) as e:
        p.select(variant=len(cands))
    assert e.value.status == -2
    with pytest.raises(st.StencilError):
        p.select(kernel=st.KERNEL_STREAM2D)


def test_fused_tiles_shrink_by_the_halo():
    p = st.Plan(synth.star_offsets(2, 1), (4096, 4096), "f32")
    by_tb = {c["tb"]: c for c in p.candidates() if c["kernel"] == st.KERNEL_STREAM2D and not c["tessellated"]}
    assert by_tb[1]["tile_x"] == 256            # 64 lanes x 4 columns, no halo
    assert by_tb[8]["tile_x"] == 256 - 2 * 8    # halo 7 rounded up to the lane width


@pytest.mark.parametrize("dtype,radius,cls,bc", [("f64", 2, "box", "zero"), ("f32", 1, "star", "periodic"),
                                                 ("f64", 1, "box", "periodic"), ("f32", 2, "star", "zero")])
def test_tessellated_candidates_geometry(dtype, radius, cls, bc):
    # Sec. 4.1's two-stage tiling: chunks of at least one junction band
    # (2R(T_b+1) rows) with no halo rows; strips as for the overlapped tiling
    # (halo R*(T_b-1) columns rounded to the lane width)
    offs = synth.star_offsets(2, radius) if cls == "star" else synth.box_offsets(2, radius)
    ny, nx = 1000, 2000
    p = st.Plan(offs, (ny, nx), dtype, bc)
    cands = p.candidates()
    tess = [c for c in cands if c["tessellated"]]
    assert tess and not cands[0]["tessellated"]     # an A/B candidate, never the default
    vx = 2 if dtype == "f64" else 4
    for c in tess:
        assert c["kernel"] == st.KERNEL_STREAM2D and 1 <= c["tb"] <= 4
        hxa = -(-radius * (c["tb"] - 1) // vx) * vx
        assert c["tile_x"] == 64 * vx - 2 * hxa
        band = 2 * radius * (c["tb"] + 1)
        assert c["tile_y"] >= band
        chunks = ny // c["tile_y"]
        assert ny - (chunks - 1) * c["tile_y"] >= c["tile_y"]   # the last chunk takes the remainder
        tiles_x = -(-nx // c["tile_x"])
        assert c["workgroups"] == -(-tiles_x * chunks // 4)
    # a grid shorter than one band: periodic plans offer none (a chunk would
    # wrap onto its own band), zero-rule plans one chunk with no junction
    ny_short = 4 * radius - 1                         # below the T_b = 1 band
    short = [c for c in st.Plan(offs, (ny_short, nx), dtype, bc).candidates() if c["tessellated"]]
    if bc == "periodic":
        assert not short
    else:
        assert short and all(c["tile_y"] == ny_short for c in short)
    # batched plans keep the overlapped tiling only
    if radius == 1:
        bp = st.BatchPlan(offs, [(64, 64), (100, 80)], dtype, bc)
        assert bp.info()["tessellated"] == 0


def _raw_plan(offsets, shape, dtype=0, bc=0, flags=0):
    lib = st.library()
    pat, keep = st._pattern(offsets)
    shp = (ctypes.c_int64 * len(shape))(*shape)
    h = ctypes.c_void_p()
    rc = lib.stencil_plan(ctypes.byref(h), ctypes.byref(pat), shp, dtype, bc, flags)
    return rc, h, keep


@pytest.mark.parametrize("offsets,shape,dtype,bc,flags,code", [
    ([(0, 0), (0, 1)], (0, 5), 0, 0, 0, -1),                 # zero extent
    ([(0, 1), (1, 0)], (5, 5), 0, 0, 0, -1),                 # no centre
    ([(0, 0), (0, 5)], (9, 9), 0, 0, 0, -2),                 # radius 5
    ([(0, 0), (0, 1), (0, 1)], (9, 9), 0, 0, 0, -1),         # repeated point
    ([(0, 0)], (9, 9), 7, 0, 0, -1),                         # bad dtype
    ([(0, 0)], (9, 9), 0, 3, 0, -1),                         # bad boundary
    ([(0, 0)], (9, 9), 0, 0, 0x80, -1),                      # unknown flag
    ([(0, 0, 0, 0)], (2, 2, 2, 2), 0, 0, 0, -2),             # 4D
])
def test_plan_rejects(offsets, shape, dtype, bc, flags, code):
    rc, h, _ = _raw_plan(offsets, shape, dtype, bc, flags)
    assert rc == code
    assert not h.value
    assert st.library().stencil_last_error()


def test_plan_rejects_null_and_too_many_points():
    lib = st.library()
    h = ctypes.c_void_p()
    shp = (ctypes.c_int64 * 2)(5, 5)
    assert lib.stencil_plan(ctypes.byref(h), None, shp, 0, 0, 0) == -1
    pat, keep = st._pattern(synth.box_offsets(3, 2) + [(3, 3, 3)])  # 126 points
    assert lib.stencil_plan(ctypes.byref(h), ctypes.byref(pat), (ctypes.c_int64 * 3)(9, 9, 9), 0, 0, 0) == -2


def test_run_rejects_bad_arguments_before_launch():
    lib = st.library()
    rc, h, keep = _raw_plan(synth.star_offsets(2, 1), (40, 50))
    assert rc == 0
    w = (ctypes.c_double * 5)(*synth.heat_weights(2, 0.1))
    good = (ctypes.c_int64 * 2)(40, 50)
    bad = (ctypes.c_int64 * 2)(40, 51)
    P = ctypes.c_void_p
    assert lib.stencil_run(h, P(FAKE), P(FAKE + 64), w, bad, 3, 0, None) == -3      # shape
    assert lib.stencil_run(h, P(FAKE), P(FAKE + 64), w, good, 3, 1, None) == -3     # boundary
    assert lib.stencil_run(h, P(FAKE), P(FAKE + 64), w, good, -1, 0, None) == -1    # steps < 0
    assert lib.stencil_run(h, None, P(FAKE), w, good, 3, 0, None) == -1             # no grid
    assert lib.stencil_run(h, P(FAKE), P(FAKE + 64), None, good, 3, 0, None) == -1  # no coeffs
    nanw = (ctypes.c_double * 5)(1.0, float("nan"), 0, 0, 0)
    assert lib.stencil_run(h, P(FAKE), P(FAKE + 64), nanw, good, 3, 0, None) == -1
    # zero steps is a no-op that touches nothing
    assert lib.stencil_run(h, P(FAKE), P(FAKE + 64), w, good, 0, 0, None) == 0
    assert lib.stencil_run(None, P(FAKE), P(FAKE + 64), w, good, 3, 0, None) == -1
    lib.stencil_plan_destroy(h)
    assert lib.stencil_plan_destroy(None) == 0


def test_run_noalloc_validation_and_work_space_limit():
    # the allocation-free run takes no work buffer; a grid beyond its 64 MiB
    # static work space is refused before anything touches the device
    lib = st.library()
    P = ctypes.c_void_p
    w7 = (ctypes.c_double * 7)(*synth.heat_weights(3, 0.1))
    big = (512, 512, 512)                       # FP64: 1 GiB
    rc, h, keep = _raw_plan(synth.star_offsets(3, 1), big)
    assert rc == 0
    shp = (ctypes.c_int64 * 3)(*big)
    assert lib.stencil_run_noalloc(h, P(FAKE), w7, shp, 3, 0, None) == -1
    assert b"static work space" in lib.stencil_last_error()
    lib.stencil_plan_destroy(h)
    # exactly 64 MiB passes the size check (256^3 FP32), one cell more fails
    for shape, dtype, ok in [((256, 256, 256), 1, True), ((256, 256, 257), 1, False),
                             ((512, 512, 128), 2, True), ((1, 1, 8 * 2 ** 20 + 1), 0, False)]:
        rc, h, keep = _raw_plan(synth.star_offsets(3, 1), shape, dtype=dtype)
        assert rc == 0
        s3 = (ctypes.c_int64 * 3)(*shape)
        # steps = 0 is a no-op once the size is accepted
        assert (lib.stencil_run_noalloc(h, P(FAKE), w7, s3, 0, 0, None) == 0) == ok, shape
        lib.stencil_plan_destroy(h)
    rc, h, keep = _raw_plan(synth.star_offsets(2, 1), (40, 50))
    w5 = (ctypes.c_double * 5)(*synth.heat_weights(2, 0.1))
    good = (ctypes.c_int64 * 2)(40, 50)
    bad = (ctypes.c_int64 * 2)(40, 51)
    assert lib.stencil_run_noalloc(None, P(FAKE), w5, good, 3, 0, None) == -1     # no plan
    assert lib.stencil_run_noalloc(h, P(FAKE), w5, bad, 3, 0, None) == -3         # shape
    assert lib.stencil_run_noalloc(h, P(FAKE), w5, good, 3, 1, None) == -3        # boundary
    assert lib.stencil_run_noalloc(h, P(FAKE), w5, good, -1, 0, None) == -1       # steps < 0
    assert lib.stencil_run_noalloc(h, None, w5, good, 3, 0, None) == -1           # no grid
    assert lib.stencil_run_noalloc(h, P(FAKE), None, good, 3, 0, None) == -1      # no coeffs
    assert lib.stencil_run_noalloc(h, P(FAKE), w5, good, 0, 0, None) == 0         # no-op
    lib.stencil_plan_destroy(h)
    bp = st.BatchPlan(synth.star_offsets(2, 1), [(8, 16)], "f32")
    assert lib.stencil_run_noalloc(bp._h, P(FAKE), w5, good, 3, 0, None) == -3    # batch plan


def test_static_work_space_is_a_file_scope_device_array_looked_up_per_device():
    # the array is never named in host code except through the symbol lookup
    src = open(os.path.join(ROOT, "paper_2303_08365_amd", "csrc", "noalloc.hip")).read()
    assert re.search(r"static __device__ __align__\(256\) unsigned char scratch\[kStaticWorkBytes\]", src)
    uses = [l for l in src.splitlines() if re.search(r"\bscratch\b", l) and not l.lstrip().startswith("//")]
    assert len(uses) == 2 and "HIP_SYMBOL(scratch)" in uses[1], uses
    abi = open(os.path.join(ROOT, "paper_2303_08365_amd", "csrc", "stencil_abi.cpp")).read()
    body = abi[abi.index("st_status stencil_run_noalloc("):]
    body = body[:body.index("\n}\n")]
    assert not re.search(r"hipMalloc|hipFree|run_graphed|hipGraph|Synchronize", body)


def test_batch_plan_and_run_validation():
    lib = st.library()
    shapes = [(37, 300), (256, 1000), (1024, 77)]
    bp = st.BatchPlan(synth.star_offsets(2, 1), shapes, "f32")
    assert bp.info()["kernel"] == st.KERNEL_STREAM2D
    P = ctypes.c_void_p
    grids = (P * 3)(FAKE, FAKE + 4096, FAKE + 8192)
    works = (P * 3)(FAKE + 64, FAKE + 4096 + 64, FAKE + 8192 + 64)
    cf = (ctypes.c_double * 15)(*(list(synth.heat_weights(2, 0.1)) * 3))
    steps = (ctypes.c_int64 * 3)(5, 5, 5)
    assert lib.stencil_batch_run(bp._h, 2, grids, works, cf, steps, None) == -3
    neg = (ctypes.c_int64 * 3)(5, -1, 5)
    assert lib.stencil_batch_run(bp._h, 3, grids, works, cf, neg, None) == -1
    same = (P * 3)(FAKE, FAKE + 4096, FAKE + 8192)
    assert lib.stencil_batch_run(bp._h, 3, grids, same, cf, steps, None) == -1
    zero = (ctypes.c_int64 * 3)(0, 0, 0)
    assert lib.stencil_batch_run(bp._h, 3, grids, works, cf, zero, None) == 0
    # 3D and general patterns are not batched
    with pytest.raises(st.StencilError):
        st.BatchPlan(synth.star_offsets(3, 1), [(8, 8)], "f32")
    with pytest.raises(st.StencilError):
        st.BatchPlan([(0, 0), (1, 2)], [(8, 8)], "f32")
    # single-grid and batch plans are not interchangeable
    rc, h, keep = _raw_plan(synth.star_offsets(2, 1), (40, 50))
    assert lib.stencil_batch_run(h, 1, grids, works, cf, steps, None) == -3
    lib.stencil_plan_destroy(h)


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device error path")
def test_run_without_device_reports_hip_error():
    lib = st.library()
    rc, h, keep = _raw_plan(synth.star_offsets(2, 1), (40, 50))
    w = (ctypes.c_double * 5)(*synth.heat_weights(2, 0.1))
    good = (ctypes.c_int64 * 2)(40, 50)
    P = ctypes.c_void_p
    assert lib.stencil_run(h, P(FAKE), P(FAKE + 64), w, good, 3, 0, None) == -5
    assert b"hipGetDeviceCount" in lib.stencil_last_error()
    lib.stencil_plan_destroy(h)


def test_varcoef_plan_and_validation():
    lib = st.library()
    p = st.varcoef_plan((16, 16, 16), "f32")
    assert p.info()["kernel"] == st.KERNEL_VARCOEF3D
    with pytest.raises(st.StencilError):
        st.Plan(synth.star_offsets(3, 1), (8, 8, 8), "f32", "periodic", varcoef=True)
    with pytest.raises(st.StencilError):
        st.Plan(synth.box_offsets(3, 1), (8, 8, 8), "f32", varcoef=True)
    with pytest.raises(st.StencilError):
        st.Plan(synth.star_offsets(3, 1), (8, 8, 8), "bf16", varcoef=True)
    P = ctypes.c_void_p
    ck = (P * 4)(FAKE, FAKE, FAKE, None)
    # plain plans cannot take a var-coef run, var-coef plans not a plain run
    q = st.Plan(synth.star_offsets(3, 1), (16, 16, 16), "f32")
    assert lib.stencil_run_ckpt(q._h, P(FAKE), P(FAKE + 64), P(FAKE), 0.1, 3, 1, None, None) == -3
    w = (ctypes.c_double * 7)(*([0.1] * 7))
    shp = (ctypes.c_int64 * 3)(16, 16, 16)
    assert lib.stencil_run(p._h, P(FAKE), P(FAKE + 64), w, shp, 3, 0, None) == -3
    assert lib.stencil_run_ckpt(p._h, P(FAKE), P(FAKE + 64), None, 0.1, 3, 1, None, None) == -1
    assert lib.stencil_run_ckpt(p._h, P(FAKE), P(FAKE + 64), P(FAKE), 0.1, 3, 0, ck, None) == -1
    assert lib.stencil_run_ckpt(p._h, P(FAKE), P(FAKE + 64), P(FAKE), 0.1, 7, 2, ck, None) == -1  # 4th NULL
    assert lib.stencil_run_ckpt(p._h, P(FAKE), P(FAKE + 64), P(FAKE), 0.1, 0, 1, None, None) == 0
    # adjoint: k required, interval >= 1, segment buffer when every > 1
    assert lib.stencil_adjoint_run(p._h, None, 0.1, None, ck, 2, 4, P(FAKE), None, P(FAKE), P(FAKE + 64), None) == -1
    assert lib.stencil_adjoint_run(p._h, P(FAKE), 0.1, None, ck, 0, 4, P(FAKE), None, P(FAKE), P(FAKE + 64), None) == -1
    assert lib.stencil_adjoint_run(p._h, P(FAKE), 0.1, None, ck, 2, 4, P(FAKE), None, None, P(FAKE + 64), None) == -1
    assert lib.stencil_adjoint_run(p._h, P(FAKE), 0.1, None, ck, 2, 0, P(FAKE), None, None, P(FAKE + 64), None) == 0
    # constant-weight adjoint refuses k / grad_k
    assert lib.stencil_adjoint_run(q._h, P(FAKE), 0.1, w, None, 0, 3, P(FAKE), None, None, P(FAKE + 64), None) == -3


def test_copy_validation():
    lib = st.library()
    P = ctypes.c_void_p
    assert lib.stencil_copy(P(FAKE), P(FAKE + 4096), 0, None) == 0
    assert lib.stencil_copy(P(FAKE), P(FAKE + 4096), -1, None) == -1
    assert lib.stencil_copy(None, P(FAKE), 64, None) == -1
    assert lib.stencil_copy(P(FAKE + 8), P(FAKE + 4096), 64, None) == -1     # misaligned
    assert lib.stencil_copy(P(FAKE), P(FAKE + 32), 64, None) == -1           # overlap


def test_library_shares_torchs_hip_runtime():
    # Loading the library before torch must not put a second libamdhip64 in
    # the process (torch's own runtime would then find no GPU).
    import subprocess
    import sys
    code = ("import paper_2303_08365_amd as st; st.library(); import torch; "
            "maps = open('/proc/self/maps').read().splitlines(); "
            "print(sorted({l.split()[-1] for l in maps if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr
    paths = eval(out.stdout.strip().splitlines()[-1])
    assert len(paths) == 1, paths


def test_3d_streaming_needs_planes_below_2gib():
    # the 3D kernel addresses a plane with 32-bit byte offsets
    import paper_2303_08365_amd as st
    offs = synth.star_offsets(3, 1)
    small = st.Plan(offs, (2, 16000, 16000), "f64")   # 2.048e9 bytes per plane
    assert any(c["kernel"] == st.KERNEL_STREAM3D for c in small.candidates())
    big = st.Plan(offs, (2, 16385, 16384), "f64")      # just above 2 GiB
    assert all(c["kernel"] == st.KERNEL_NAIVE for c in big.candidates())
    assert big.info()["kernel"] == st.KERNEL_NAIVE


def test_autotune_cache_file_validation(tmp_path):
    import paper_2303_08365_amd as st
    bad = tmp_path / "bad.txt"
    bad.write_text("v1 some key\t3\n")
    with pytest.raises(st.StencilError):
        st.autotune_cache(str(bad))
    bad.write_text("v1 some key\t5\t4\n")  # candidate outside 0..3
    with pytest.raises(st.StencilError):
        st.autotune_cache(str(bad))
    good = tmp_path / "good.txt"
    good.write_text("v1 dev nd3 t0 bc0 grid 8x8x8 p 0,0,0\t1\t4\n\n")
    st.autotune_cache(str(good))
    st.autotune_cache(str(tmp_path / "missing.txt"))  # created on the first tuning
    st.autotune_cache(None)
    with pytest.raises(st.StencilError):
        st.autotune_cache("")


def test_binding_refuses_host_tensors_and_short_adjoint_buffers():
    # every tensor the kernels touch must be GPU memory: a host pointer would
    # reach a kernel; the adjoint's checkpoint list and segment buffer are
    # sized before the call (the C side reads ceil(steps/every) pointers)
    import torch
    shp = (4, 8, 16)
    cpu = torch.zeros(shp, dtype=torch.float64)
    p = st.Plan(synth.star_offsets(3, 1), shp, "f64")
    w = list(synth.heat_weights(3, 0.1))
    with pytest.raises(ValueError, match="GPU tensor"):
        p.run(cpu, w, 2)
    with pytest.raises(ValueError, match="GPU tensor"):
        p.run_flux(cpu, w, 2, torch.zeros(1, dtype=torch.float64))
    with pytest.raises(ValueError, match="GPU tensor"):
        p.run_noalloc(cpu, w, 2)
    with pytest.raises(ValueError, match="GPU tensor"):
        p.adjoint(cpu.clone(), 2, cpu.clone(), coeffs=w)
    with pytest.raises(ValueError, match="GPU tensor"):
        st.copy(cpu.clone(), cpu)
    vp = st.Plan(synth.star_offsets(3, 1), shp, "f64", varcoef=True)
    with pytest.raises(ValueError, match="GPU tensor"):
        vp.run_ckpt(cpu.clone(), cpu.clone(), 0.1, 4, cpu.clone(), every=2, ckpts=[cpu.clone(), cpu.clone()])
    with pytest.raises(ValueError, match="checkpoint tensors are required"):
        vp.run_ckpt(cpu.clone(), cpu.clone(), 0.1, 4, cpu.clone(), every=2, ckpts=[cpu.clone()])
    with pytest.raises(ValueError, match="checkpoint tensors are required"):
        vp.adjoint(cpu.clone(), 10, cpu.clone(), k=cpu.clone(), alpha=0.1, ckpts=[cpu.clone()] * 2, every=4,
                   seg=torch.zeros((3,) + shp, dtype=torch.float64))
    with pytest.raises(ValueError, match="every must be >= 1"):
        vp.adjoint(cpu.clone(), 10, cpu.clone(), k=cpu.clone(), alpha=0.1, ckpts=[cpu.clone()] * 3, every=0)
    with pytest.raises(ValueError, match="seg must hold"):
        vp.adjoint(cpu.clone(), 10, cpu.clone(), k=cpu.clone(), alpha=0.1, ckpts=[cpu.clone()] * 3, every=4)
    with pytest.raises(ValueError, match="seg holds"):
        vp.adjoint(cpu.clone(), 10, cpu.clone(), k=cpu.clone(), alpha=0.1, ckpts=[cpu.clone()] * 3, every=4,
                   seg=torch.zeros((2,) + shp, dtype=torch.float64))
    with pytest.raises(ValueError, match="plan's shape"):
        vp.adjoint(cpu.clone(), 10, cpu.clone(), k=cpu.clone(), alpha=0.1,
                   ckpts=[cpu.clone(), cpu.clone(), torch.zeros((4, 8, 8), dtype=torch.float64)], every=4,
                   seg=torch.zeros((3,) + shp, dtype=torch.float64))
    with pytest.raises(ValueError, match="GPU tensor"):
        vp.adjoint(cpu.clone(), 10, cpu.clone(), k=cpu.clone(), alpha=0.1, ckpts=[cpu.clone()] * 3, every=4,
                   seg=torch.zeros((3,) + shp, dtype=torch.float64))
    bp = st.BatchPlan(synth.star_offsets(2, 1), [(8, 16), (9, 16)], "f32")
    g = [torch.zeros(s, dtype=torch.float32) for s in [(8, 16), (9, 16)]]
    with pytest.raises(ValueError, match="GPU tensor"):
        bp.run(g, [x.clone() for x in g], [list(synth.heat_weights(2, 0.1, "f32"))] * 2, [2, 2])


def _enclosing_functions(src, pattern):
    """Names of the top-level functions of `src` whose bodies contain `pattern`
    (a function starts at a column-0 line holding `name(` and ends at the
    next column-0 `}`)."""
    found = set()
    current = None
    for line in src.splitlines():
        m = re.match(r"^[A-Za-z_][\w:<>,\s\*&]*?\b(\w+)\s*\(", line)
        if m and not line.startswith(("#", "//", "namespace", "extern", "struct", "using", "template", "typedef")):
            current = m.group(1)
        if line.startswith("}"):
            pass
        if re.search(pattern, line) and not line.lstrip().startswith("//"):
            found.add(current)
    return found


def test_run_calls_neither_allocate_nor_wait():
    # every device allocation, free, stream creation and host wait of the
    # library sits in plan creation, autotuning or plan destruction: no run
    # entry point (stencil_run, _flux, _batch_run, _ckpt, _adjoint) reaches one
    src = open(os.path.join(ROOT, "paper_2303_08365_amd", "csrc", "stencil_abi.cpp")).read()
    allowed = {"plan_buffers", "autotune", "batch_autotune", "stencil_plan_destroy"}
    for pat in (r"\bhipMalloc\w*\s*\(", r"\bhipHostMalloc\s*\(", r"\bhipFree\w*\s*\(", r"\bhipHostFree\s*\(",
                r"Synchronize\s*\(", r"\bhipStreamCreate\w*\s*\(", r"\bhipEventCreate\w*\s*\(",
                r"\bhipMallocAsync\s*\("):
        where = _enclosing_functions(src, pat)
        assert where <= allowed, (pat, where - allowed)
    assert "ST_ERR_CAPTURE" not in src


def _gpu_code_objects(so_path):
    """The gfx950 code objects bundled into the library's .hip_fatbin section
    (one clang offload bundle per translation unit)."""
    readelf = "/opt/rocm/llvm/bin/llvm-readelf"
    out = subprocess.run([readelf, "-S", "-W", so_path], capture_output=True, text=True, check=True).stdout
    off = size = None
    for line in out.splitlines():
        if ".hip_fatbin" in line:
            f = line.split("]", 1)[1].split()
            off, size = int(f[3], 16), int(f[4], 16)
    assert off is not None, "no .hip_fatbin section"
    with open(so_path, "rb") as fh:
        fh.seek(off)
        data = fh.read(size)
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    objs, pos = [], 0
    while True:
        i = data.find(magic, pos)
        if i < 0:
            return objs
        n = struct.unpack_from("<Q", data, i + len(magic))[0]
        p = i + len(magic) + 8
        for _ in range(n):
            o, s, ts = struct.unpack_from("<QQQ", data, p)
            p += 24
            triple = data[p:p + ts].decode()
            p += ts
            if "amdgcn" in triple and s > 0:
                objs.append(data[i + o:i + o + s])
        pos = i + len(magic)


def test_lds_queue_kernels_keep_their_memory_count():
    # The 7-point pipeline's LDS-queue form reads its queue slot after an
    # explicit wait that counts the memory operations of one iteration (K + 1
    # queue loads, K stores).  A register spill would add scratch operations
    # to that count: every such kernel must use no scratch, and must load
    # through the queue (buffer loads into LDS).
    import re
    objdump = "/opt/rocm/llvm/bin/llvm-objdump"
    if not os.path.exists(objdump):
        pytest.skip("llvm-objdump is not installed")
    found = 0
    with tempfile.TemporaryDirectory() as d:
        for k, b in enumerate(_gpu_code_objects(st.library_path())):
            f = os.path.join(d, f"co{k}.o")
            with open(f, "wb") as fh:
                fh.write(b)
            dis = subprocess.run([objdump, "-d", f], capture_output=True, text=True, check=True).stdout
            for m in re.finditer(r"^[0-9a-f]+ <(_Z\w*pipe3d_kernel\w*ELb1EEEvNS_12Stream3DArgsE)>:\n(.*?)(?=^[0-9a-f]+ <|\Z)",
                                 dis, re.S | re.M):
                name, body = m.group(1), m.group(2)
                found += 1
                assert "scratch_" not in body, f"{name} spills to scratch"
                assert re.search(r"buffer_load_dwordx4 .* lds", body), f"{name} has no queue loads"
    assert found >= 4, "no LDS-queue kernel in the library"


def test_box_pipeline_kernels_do_not_spill():
    # The 27-point box pipeline carries two levels' planes and partial sums in
    # registers (225-250 VGPRs at 2 waves per SIMD); the forms that spill
    # (more rows a lane, the copy-free unrolled loops) measured far slower,
    # so every instance in the library must use no scratch.
    import re
    objdump = "/opt/rocm/llvm/bin/llvm-objdump"
    if not os.path.exists(objdump):
        pytest.skip("llvm-objdump is not installed")
    found = 0
    with tempfile.TemporaryDirectory() as d:
        for k, b in enumerate(_gpu_code_objects(st.library_path())):
            f = os.path.join(d, f"co{k}.o")
            with open(f, "wb") as fh:
                fh.write(b)
            dis = subprocess.run([objdump, "-d", f], capture_output=True, text=True, check=True).stdout
            for m in re.finditer(r"^[0-9a-f]+ <(_Z\w*boxpipe3d_kernel\w*)>:\n(.*?)(?=^[0-9a-f]+ <|\Z)", dis, re.S | re.M):
                name, body = m.group(1), m.group(2)
                found += 1
                assert "scratch_" not in body, f"{name} spills to scratch"
                assert "s_barrier" in body, f"{name} has no barrier"
    assert found >= 4, "no box pipeline kernel in the library"


def test_kernels_contain_no_device_function_calls():
    # Every kernel is inlined into one function that ends in s_endpgm: no
    # device-function call, hence no return address.  An earlier build
    # outlined the bfloat16 radius-2 2D body into a call; the compiler's
    # long-branch expansion in that function reused the return-address pair
    # s[30:31], and waves leaving early through that branch (work items past
    # the item count) then "returned" into their own branch target forever.
    objdump = "/opt/rocm/llvm/bin/llvm-objdump"
    if not os.path.exists(objdump):
        pytest.skip("llvm-objdump is not installed")
    objs = _gpu_code_objects(st.library_path())
    assert len(objs) >= 10
    with tempfile.TemporaryDirectory() as d:
        for k, b in enumerate(objs):
            f = os.path.join(d, f"co{k}.o")
            with open(f, "wb") as fh:
                fh.write(b)
            dis = subprocess.run([objdump, "-d", f], capture_output=True, text=True, check=True).stdout
            assert "s_swappc_b64" not in dis, f"code object {k} contains a device-function call"
            assert "s_setpc_b64 s[30:31]" not in dis, f"code object {k} jumps through the return-address pair"
