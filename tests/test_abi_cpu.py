"""The C ABI on the CPU: the library loads, exports every declared symbol, and rejects
bad arguments on the host before any HIP call (so none of this needs a GPU)."""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

import paper_1810_03988_amd as P
from paper_1810_03988_amd import stitch as S
import workloads as wl

HEADER = Path(__file__).resolve().parents[1] / "include" / "stitch.h"
E = {name: i for i, name in enumerate(S.STATUS)}


def declared_symbols():
    text = re.sub(r"/\*.*?\*/", "", HEADER.read_text(), flags=re.S)
    return sorted(set(re.findall(r"\b(stitch_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    names = declared_symbols()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
        assert n in S.SIGNATURES, f"{n} has no binding"
    assert lib.stitch_abi_version() == 1
    assert lib.stitch_status_str(5) == b"invalid seam weights"


def _plan_args(rig=None, masks=None, levels=None, storage=S.F32, H=None):
    rig = rig or wl.rig_c1()
    n = rig.n
    masks = masks if masks is not None else rig.masks()
    fw = (ctypes.c_int32 * n)(*[s[0] for s in rig.frame_sizes])
    fh = (ctypes.c_int32 * n)(*[s[1] for s in rig.frame_sizes])
    Hs = np.ascontiguousarray(np.stack([np.asarray(h, float).reshape(9) for h in (H or rig.H)]))
    keep = [np.ascontiguousarray(m) for m in masks]
    mp = (ctypes.POINTER(ctypes.c_uint8) * n)(*[m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) for m in keep])
    return (n, fw, fh, Hs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mp, rig.canvas_w, rig.canvas_h,
            levels or rig.levels, storage, 0), (keep, Hs)


def _create(*args):
    h = ctypes.c_void_p()
    st = P.lib().stitch_plan_create(*args, ctypes.byref(h))
    return st, h


def test_plan_create_and_regions_are_aligned():
    args, keep = _plan_args()
    st, h = _create(*args)
    assert st == 0, P.stitch.last_error()
    try:
        assert P.lib().stitch_plan_workspace_bytes(h) > 0
        L = args[7]
        for cam in range(2):
            roi = (ctypes.c_int32 * 4)()
            band = (ctypes.c_int32 * 4)()
            for k in range(L):
                assert P.lib().stitch_plan_regions(h, cam, k, roi, band) == 0
                if k == 0:
                    assert roi[0] % (1 << (L - 1)) == 0 and roi[1] % (1 << (L - 1)) == 0
                # the band window lies inside the roi
                assert band[0] >= roi[0] and band[0] + band[2] <= roi[0] + roi[2]
                assert band[1] >= roi[1] and band[1] + band[3] <= roi[1] + roi[3]
        # camera B's footprint starts near x = 392 and its seam weights at x = 520: its roi
        # covers what the blend reads of it (the band plus the pyramid's reach), not the
        # whole footprint and not the canvas edge
        assert P.lib().stitch_plan_regions(h, 1, 0, roi, band) == 0
        assert 392 - 32 < roi[0] <= band[0] - 32 and band[0] == 520
    finally:
        P.lib().stitch_plan_destroy(h)


@pytest.mark.parametrize("case,code", [
    ("mask_sum", "E_MASK"), ("levels_deep", "E_LEVELS"), ("levels_zero", "E_LEVELS"), ("nan_h", "E_HOMOGRAPHY"),
    ("singular_h", "E_HOMOGRAPHY"), ("storage", "E_UNSUPPORTED"), ("null_mask", "E_NULL"),
])
def test_plan_create_rejects(case, code):
    rig = wl.rig_c1()
    kw = {}
    if case == "mask_sum":
        kw["masks"] = [rig.masks()[0], rig.masks()[0]]
    elif case == "levels_deep":
        kw["levels"] = 9          # 480 -> ... -> 2 at level 8
    elif case == "levels_zero":
        kw["levels"] = 17
    elif case == "nan_h":
        H = [h.copy() for h in rig.H]
        H[1][0, 2] = np.nan
        kw["H"] = H
    elif case == "singular_h":
        H = [h.copy() for h in rig.H]
        H[1][:2, :2] = [[1.0, 2.0], [2.0, 4.0]]
        kw["H"] = H
    elif case == "storage":
        kw["storage"] = 7
    args, keep = _plan_args(rig, **kw)
    if case == "null_mask":
        args = list(args)
        mp = (ctypes.POINTER(ctypes.c_uint8) * 2)(args[4][0], ctypes.POINTER(ctypes.c_uint8)())
        args[4] = mp
    st, h = _create(*args)
    assert st == E[code], (st, P.stitch.last_error())
    assert not h.value
    assert len(P.stitch.last_error()) > 0


def test_frame_requires_bound_workspace_and_valid_views():
    args, keep = _plan_args()
    st, h = _create(*args)
    assert st == 0
    try:
        fake = 0x10000
        frames = (S.StitchImage * 2)(S.StitchImage(fake, 640, 480, 3, S.U8, S.HWC, 1920, 0),
                                     S.StitchImage(fake, 640, 480, 3, S.U8, S.HWC, 1920, 0))
        pano = S.StitchImage(fake, 1040, 480, 3, S.U8, S.HWC, 3120, 0)
        assert P.lib().stitch_frame(h, frames, ctypes.byref(pano), None) == E["E_STATE"]
        assert P.lib().stitch_frame(h, None, ctypes.byref(pano), None) == E["E_NULL"]
        assert P.lib().stitch_plan_bind(h, None, 0, None) == E["E_WORKSPACE"]
        assert P.lib().stitch_plan_bind(h, 0x10001, 1 << 40, None) == E["E_WORKSPACE"]   # misaligned
        assert P.lib().stitch_plan_bind(h, 0x10000, 16, None) == E["E_WORKSPACE"]        # too small
    finally:
        P.lib().stitch_plan_destroy(h)


def test_single_stage_calls_validate_on_host():
    lib = P.lib()
    fake = 0x10000
    H = (ctypes.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    Hbad = (ctypes.c_double * 9)(1, 2, 0, 2, 4, 0, 0, 0, 1)
    src = S.StitchImage(fake, 64, 48, 3, S.U8, S.HWC, 192, 0)
    dst = S.StitchImage(fake, 64, 48, 3, S.F32, S.CHW, 256, 256 * 48)
    assert lib.stitch_warp(None, H, 0, 0, ctypes.byref(dst), None) == E["E_NULL"]
    assert lib.stitch_warp(ctypes.byref(src), Hbad, 0, 0, ctypes.byref(dst), None) == E["E_HOMOGRAPHY"]
    bad = S.StitchImage(fake, 64, 48, 3, S.U8, S.CHW, 64, 64 * 48)
    assert lib.stitch_warp(ctypes.byref(src), H, 0, 0, ctypes.byref(bad), None) == E["E_UNSUPPORTED"]
    short = S.StitchImage(fake, 64, 48, 3, S.F32, S.CHW, 100, 256 * 48)
    assert lib.stitch_warp(ctypes.byref(src), H, 0, 0, ctypes.byref(short), None) == E["E_SHAPE"]
    # pyramid: a level side below 3 is rejected before anything runs
    lv = S.StitchLevels()
    lv.levels, lv.canvas_w, lv.canvas_h = 3, 8, 8
    for k, s in enumerate([8, 4, 2]):
        lv.level[k] = S.StitchImage(fake, s, s, 1, S.F32, S.CHW, 256, 256 * s)
    g0 = S.StitchImage(fake, 8, 8, 1, S.F32, S.CHW, 256, 2048)
    assert lib.stitch_pyramid(ctypes.byref(g0), 1, ctypes.byref(lv), fake, 4096, None) == E["E_LEVELS"]
    lv.levels = 2
    assert lib.stitch_pyramid(ctypes.byref(g0), 1, ctypes.byref(lv), None, 0, None) == E["E_WORKSPACE"]
    assert lib.stitch_pyramid(ctypes.byref(g0), 3, ctypes.byref(lv), fake, 4096, None) == E["E_UNSUPPORTED"]
    # the kernels address a level with 32-bit offsets: rows of 2^23 elements or more are refused
    lv.level[1] = S.StitchImage(fake, 4, 4, 1, S.F32, S.CHW, (1 << 23) * 4, (1 << 23) * 16)
    assert lib.stitch_pyramid(ctypes.byref(g0), 1, ctypes.byref(lv), fake, 4096, None) == E["E_SHAPE"]
    lv.level[1] = S.StitchImage(fake, 4, 4, 1, S.F32, S.CHW, 256, 256 * 4)
    # blend: missing R storage for a multi-level blend
    pano = S.StitchImage(fake, 8, 8, 3, S.U8, S.HWC, 24, 0)
    b = S.StitchLevels()
    b.levels, b.canvas_w, b.canvas_h = 2, 8, 8
    w = S.StitchLevels()
    w.levels, w.canvas_w, w.canvas_h = 2, 8, 8
    for k, s in enumerate([8, 4]):
        b.level[k] = S.StitchImage(fake, s, s, 3, S.F32, S.CHW, 256, 256 * s)
        w.level[k] = S.StitchImage(fake, s, s, 1, S.F32, S.CHW, 256, 256 * s)
    assert lib.stitch_blend(1, ctypes.byref(b), ctypes.byref(w), ctypes.byref(pano), None, fake, 1 << 20,
                            None) == E["E_NULL"]
    assert lib.stitch_blend(0, ctypes.byref(b), ctypes.byref(w), ctypes.byref(pano), None, fake, 1 << 20,
                            None) == E["E_SHAPE"]
    # three band planes spanning 2^31 elements or more are refused (32-bit offsets)
    b.level[1] = S.StitchImage(fake, 4, 4, 3, S.F32, S.CHW, 256, (1 << 30) * 4)
    assert lib.stitch_blend(1, ctypes.byref(b), ctypes.byref(w), ctypes.byref(pano), None, fake, 1 << 20,
                            None) == E["E_SHAPE"]


def test_pipe_validates_on_host():
    lib = P.lib()
    args, keep = _plan_args()
    st, h = _create(*args)
    assert st == 0
    try:
        out = ctypes.c_void_p()
        fake = 0x10000
        # slots: each frame set and panorama, every buffer rounded up to 256 bytes
        slot = sum(-(-w * hh * 3 // 256) * 256 for w, hh in wl.rig_c1().frame_sizes) + -(-1040 * 480 * 3 // 256) * 256
        need = lib.stitch_pipe_workspace_bytes(h, 2)
        assert need == 2 * slot
        assert lib.stitch_pipe_workspace_bytes(h, 0) == 0 and lib.stitch_pipe_workspace_bytes(None, 2) == 0
        assert lib.stitch_pipe_create(None, 2, fake, need, ctypes.byref(out)) == E["E_NULL"]
        assert lib.stitch_pipe_create(h, 0, fake, need, ctypes.byref(out)) == E["E_SHAPE"]
        assert lib.stitch_pipe_create(h, 9, fake, need, ctypes.byref(out)) == E["E_SHAPE"]
        assert lib.stitch_pipe_create(h, 2, None, need, ctypes.byref(out)) == E["E_WORKSPACE"]
        assert lib.stitch_pipe_create(h, 2, fake + 16, need, ctypes.byref(out)) == E["E_WORKSPACE"]
        assert lib.stitch_pipe_create(h, 2, fake, need - 1, ctypes.byref(out)) == E["E_WORKSPACE"]
        assert lib.stitch_pipe_create(h, 2, fake, need, ctypes.byref(out)) == E["E_STATE"]   # no workspace bound
        assert out.value is None
        assert lib.stitch_pipe_run(None, 1, None, None) == E["E_NULL"]
        assert lib.stitch_host_alloc(16, None) == E["E_NULL"]
        lib.stitch_pipe_destroy(None)
        lib.stitch_host_free(None)
    finally:
        lib.stitch_plan_destroy(h)


def test_lorb_validates_on_host():
    lib = P.lib()
    fake = 0x10000
    frame = S.StitchImage(fake, 640, 480, 3, S.U8, S.HWC, 1920, 0)
    areas = (ctypes.c_int32 * 8)(0, 0, 300, 200, 100, 50, 80, 80)
    bad_areas = (ctypes.c_int32 * 8)(0, 0, 300, 200, 100, 50, -1, 80)
    outs = [fake] * 4

    def call(fr=ctypes.byref(frame), m=2, ar=areas, tf=20, t=0, n=500, nd=256, pat=fake, o=outs):
        return lib.stitch_lorb(fr, m, ar, tf, t, n, nd, pat, *o, fake, 1 << 30, None)

    assert call(fr=None) == E["E_NULL"]
    assert call(pat=None) == E["E_NULL"]
    assert call(o=[fake, None, fake, fake]) == E["E_NULL"]
    assert call(m=0) == E["E_SHAPE"] and call(m=65) == E["E_SHAPE"]
    for nd in (0, 16, 48, 544):
        assert call(nd=nd) == E["E_SHAPE"], nd
    assert call(n=0) == E["E_SHAPE"] and call(n=(1 << 20) + 1) == E["E_SHAPE"]
    assert call(tf=-1) == E["E_SHAPE"] and call(tf=256) == E["E_SHAPE"]
    assert call(ar=bad_areas) == E["E_SHAPE"]
    tiny = S.StitchImage(fake, 34, 480, 3, S.U8, S.HWC, 102, 0)
    assert call(fr=ctypes.byref(tiny)) == E["E_SHAPE"]           # no sample 17 from both sides
    chw = S.StitchImage(fake, 640, 480, 3, S.U8, S.CHW, 640, 640 * 480)
    assert call(fr=ctypes.byref(chw)) != 0
    gray = S.StitchImage(fake, 640, 480, 1, S.U8, S.HWC, 640, 0)
    assert call(fr=ctypes.byref(gray)) == E["E_SHAPE"]
    assert lib.stitch_lorb_workspace_bytes(640, 480, 0, areas) == 0
    assert lib.stitch_lorb_workspace_bytes(640, 480, 2, bad_areas) == 0
    # 24 bytes per sample of the clipped areas (283 x 183 and 80 x 80), counters and padding
    need = lib.stitch_lorb_workspace_bytes(640, 480, 2, areas)
    base = 24 * (283 * 183 + 80 * 80)
    assert base <= need < base + 4096
    assert call(pat=fake + 4) == E["E_SHAPE"]                    # pattern not 16-byte aligned
    assert lib.stitch_lorb(ctypes.byref(frame), 2, areas, 20, 0, 500, 256, fake, *outs, fake, need - 1,
                           None) == E["E_WORKSPACE"]
    assert lib.stitch_lorb(ctypes.byref(frame), 2, areas, 20, 0, 500, 256, fake, *outs, fake + 64, need,
                           None) == E["E_WORKSPACE"]


def test_lorb_multi_validates_on_host():
    lib = P.lib()
    fake = 0x10000
    imgs = (S.StitchImage * 2)(S.StitchImage(fake, 640, 480, 3, S.U8, S.HWC, 1920, 0),
                               S.StitchImage(fake, 320, 240, 3, S.U8, S.HWC, 960, 0))
    fw, fh = (ctypes.c_int32 * 2)(640, 320), (ctypes.c_int32 * 2)(480, 240)
    areas = (ctypes.c_int32 * 12)(0, 0, 300, 200, 100, 50, 80, 80, 10, 10, 100, 100)
    mpf = (ctypes.c_int32 * 2)(2, 1)
    outs = [fake] * 4

    def call(n=2, im=imgs, m=mpf, ar=areas):
        return lib.stitch_lorb_multi(n, im, m, ar, 20, 0, 500, 256, fake, *outs, fake, 1 << 30, None)

    assert call(im=None) == E["E_NULL"] and call(m=None) == E["E_NULL"]
    assert call(n=0) == E["E_SHAPE"] and call(n=17) == E["E_SHAPE"]
    assert call(m=(ctypes.c_int32 * 2)(2, -1)) == E["E_SHAPE"]
    assert call(m=(ctypes.c_int32 * 2)(0, 0)) == E["E_SHAPE"]              # no area at all
    # 24 bytes per scanned sample: 283 x 183 and 80 x 80 in the first frame, 93 x 93 in the second
    need = lib.stitch_lorb_multi_workspace_bytes(2, fw, fh, mpf, areas)
    base = 24 * (283 * 183 + 80 * 80 + 93 * 93)
    assert base <= need < base + 4096
    assert lib.stitch_lorb_multi_workspace_bytes(2, fw, fh, (ctypes.c_int32 * 2)(0, 0), areas) == 0


def test_registration_calls_validate_on_host():
    lib = P.lib()
    fake = 0x10000
    pos = (ctypes.c_int32 * 24)(*range(24))
    bad_pos = (ctypes.c_int32 * 24)(*([3] * 23 + [256]))

    def match(nd=256, a=fake, cap_a=100, cap_b=100, tables=2, kbits=12, p=pos, ws=fake, nbytes=1 << 20):
        return lib.stitch_lsh_match(nd, a, fake, cap_a, fake, fake, cap_b, tables, kbits, p, 64, fake, fake, ws,
                                    nbytes, None)

    assert match(a=None) == E["E_NULL"]
    assert match(p=None) == E["E_NULL"] and match(p=None, kbits=0) != E["E_NULL"]
    assert match(nd=48) == E["E_SHAPE"] and match(cap_a=0) == E["E_SHAPE"] and match(cap_b=65537) == E["E_SHAPE"]
    assert match(tables=17) == E["E_SHAPE"] and match(kbits=25) == E["E_SHAPE"]
    assert match(p=bad_pos) == E["E_SHAPE"]                      # a bit position past nd
    assert match(a=fake + 4) == E["E_SHAPE"]                     # descriptors not 8-byte aligned
    need = lib.stitch_lsh_match_workspace_bytes(100, 100, 2)
    assert need >= 2 * 100 * 4 * 2
    assert match(ws=fake + 16) == E["E_WORKSPACE"] and match(nbytes=need - 1) == E["E_WORKSPACE"]
    assert lib.stitch_lsh_match_workspace_bytes(0, 100, 2) == 0

    def prosac(pa=fake, cap_a=100, nhyp=512, T_N=2e5, eps=3.0, nbytes=1 << 24, ws=fake):
        return lib.stitch_prosac(pa, fake, 100, fake, fake, fake, cap_a, nhyp, fake, T_N, eps, fake, fake, fake,
                                 fake, ws, nbytes, None)

    assert prosac(pa=None) == E["E_NULL"]
    assert prosac(nhyp=0) == E["E_SHAPE"] and prosac(nhyp=65537) == E["E_SHAPE"]
    assert prosac(T_N=0.0) == E["E_SHAPE"] and prosac(eps=float("nan")) == E["E_SHAPE"]
    assert prosac(T_N=2.0 ** 53 * 1.5) == E["E_SHAPE"] and prosac(T_N=float("inf")) == E["E_SHAPE"]
    assert prosac(cap_a=70000) == E["E_SHAPE"]
    need = lib.stitch_prosac_workspace_bytes(100, 512)
    assert need >= 512 * 9 * 8
    assert prosac(nbytes=need - 1) == E["E_WORKSPACE"] and prosac(ws=fake + 8) == E["E_WORKSPACE"]


def test_multi_pair_registration_calls_validate_on_host():
    """stitch_lsh_match_multi / stitch_prosac_multi: workspace = a table head plus each
    pair's single-pair workspace (which also pins the pair structs' field offsets), and every
    argument check, per pair, before anything reaches the device."""
    lib = P.lib()
    fake = 0x10000
    pos = (ctypes.c_int32 * 24)(*range(24))
    caps = [(10, 20), (500, 300), (7, 7)]

    def mpairs(**over):
        t = (S.MatchPair * 3)()
        for p, (a, b) in enumerate(caps):
            t[p] = S.MatchPair(fake, fake, a, fake, fake, b, fake, fake)
        for k, v in over.items():
            setattr(t[1], k, v)
        return t

    single = sum(lib.stitch_lsh_match_workspace_bytes(a, b, 2) for a, b in caps)
    need = lib.stitch_lsh_match_multi_workspace_bytes(3, mpairs(), 2)
    assert single < need <= single + 4096
    assert lib.stitch_lsh_match_multi_workspace_bytes(0, mpairs(), 2) == 0
    assert lib.stitch_lsh_match_multi_workspace_bytes(257, mpairs(), 2) == 0
    assert lib.stitch_lsh_match_multi_workspace_bytes(3, mpairs(cap_b=0), 2) == 0

    def match(t=None, n=3, nd=256, tables=2, kbits=12, p=pos, ws=fake, nbytes=need):
        return lib.stitch_lsh_match_multi(n, mpairs() if t is None else t, nd, tables, kbits, p, 64, ws, nbytes,
                                          None)

    assert lib.stitch_lsh_match_multi(3, None, 256, 2, 12, pos, 64, fake, need, None) == E["E_NULL"]
    assert match(p=None) == E["E_NULL"]
    assert match(t=mpairs(desc_b=None)) == E["E_NULL"] and "pair 1" in S.last_error()
    assert match(t=mpairs(dist=None)) == E["E_NULL"]
    assert match(n=0) == E["E_SHAPE"] and match(n=257) == E["E_SHAPE"]
    assert match(nd=48) == E["E_SHAPE"] and match(tables=17) == E["E_SHAPE"] and match(kbits=25) == E["E_SHAPE"]
    assert match(t=mpairs(cap_a=0)) == E["E_SHAPE"] and match(t=mpairs(cap_b=65537)) == E["E_SHAPE"]
    assert match(t=mpairs(desc_a=fake + 4)) == E["E_SHAPE"] and "pair 1" in S.last_error()
    assert match(ws=None) == E["E_WORKSPACE"] and match(ws=fake + 16) == E["E_WORKSPACE"]
    assert match(nbytes=need - 1) == E["E_WORKSPACE"]

    def ppairs(**over):
        t = (S.ProsacPair * 3)()
        for p, (a, b) in enumerate(caps):
            t[p] = S.ProsacPair(fake, fake, b, fake, fake, fake, a, fake, fake, fake, fake, fake)
        for k, v in over.items():
            setattr(t[2], k, v)
        return t

    single = sum(lib.stitch_prosac_workspace_bytes(a, 512) for a, _ in caps)
    pneed = lib.stitch_prosac_multi_workspace_bytes(3, ppairs(), 512)
    assert single < pneed <= single + 4096
    assert lib.stitch_prosac_multi_workspace_bytes(3, ppairs(), 0) == 0
    assert lib.stitch_prosac_multi_workspace_bytes(3, ppairs(cap_a=70000), 512) == 0

    def prosac(t=None, n=3, nhyp=512, T_N=2e5, eps=3.0, ws=fake, nbytes=pneed):
        return lib.stitch_prosac_multi(n, ppairs() if t is None else t, nhyp, T_N, eps, ws, nbytes, None)

    assert lib.stitch_prosac_multi(3, None, 512, 2e5, 3.0, fake, pneed, None) == E["E_NULL"]
    assert prosac(t=ppairs(uniforms=None)) == E["E_NULL"] and "pair 2" in S.last_error()
    assert prosac(t=ppairs(hyp_counts=None)) == E["E_NULL"]
    assert prosac(n=0) == E["E_SHAPE"] and prosac(n=257) == E["E_SHAPE"]
    assert prosac(nhyp=0) == E["E_SHAPE"] and prosac(nhyp=65537) == E["E_SHAPE"]
    assert prosac(T_N=0.0) == E["E_SHAPE"] and prosac(eps=float("inf")) == E["E_SHAPE"]
    assert prosac(T_N=2.0 ** 53 * 1.5) == E["E_SHAPE"]
    assert prosac(t=ppairs(cap_a=0)) == E["E_SHAPE"] and prosac(t=ppairs(cap_b=65537)) == E["E_SHAPE"]
    assert prosac(ws=None) == E["E_WORKSPACE"] and prosac(ws=fake + 8) == E["E_WORKSPACE"]
    assert prosac(nbytes=pneed - 1) == E["E_WORKSPACE"]


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(S, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(S, "_lib", None)
    with pytest.raises(ImportError):
        S.lib()


def test_batch_group_calls_validate_on_host():
    lib = P.lib()
    assert lib.stitch_batch_set_groups(None, 2) == E["E_NULL"]
    assert lib.stitch_batch_group_count(None) == 0


def test_batch_create_validates_on_host():
    lib = P.lib()
    args, keep = _plan_args()
    st, h = _create(*args)
    assert st == 0
    try:
        out = ctypes.c_void_p()
        arr = (ctypes.c_void_p * 1)(h.value)
        assert lib.stitch_batch_create(1, arr, ctypes.byref(out)) == E["E_STATE"]   # not bound
        assert lib.stitch_batch_create(0, arr, ctypes.byref(out)) == E["E_SHAPE"]
        assert lib.stitch_batch_create(1, None, ctypes.byref(out)) == E["E_NULL"]
        assert not out.value
    finally:
        lib.stitch_plan_destroy(h)


def _grad_create(masks, W, H, L, fw=(64, 64), fh=(48, 48)):
    ms = [np.ascontiguousarray(m) for m in masks]
    mp = (ctypes.POINTER(ctypes.c_uint8) * 2)(*[m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) for m in ms])
    h = ctypes.c_void_p()
    st = P.lib().stitch_grad_create((ctypes.c_int32 * 2)(*fw), (ctypes.c_int32 * 2)(*fh), mp, W, H, L,
                                    ctypes.byref(h))
    return st, h


def test_grad_form_validates_on_host():
    lib = P.lib()
    W, H = 96, 48
    m0 = np.zeros((H, W), np.uint8)
    m0[:, : W // 2] = 255
    good = [m0, 255 - m0]
    st, h = _grad_create(good, W, H, 3)
    assert st == 0, S.last_error()
    try:
        assert lib.stitch_grad_workspace_bytes(h) > 0
        H18 = (ctypes.c_double * 18)(*np.tile(np.eye(3).ravel(), 2))
        # freeze / forward / backward before bind
        assert lib.stitch_grad_freeze(h, H18, None, None) == E["E_STATE"]
        loss = ctypes.c_double()
        assert lib.stitch_grad_forward(h, (S.StitchImage * 2)(), H18, ctypes.byref(loss), None) == E["E_STATE"]
        assert lib.stitch_grad_backward(h, (S.StitchImage * 2)(), (ctypes.c_double * 18)(), None) == E["E_STATE"]
        # bind with no or misaligned memory
        assert lib.stitch_grad_bind(h, None, 1 << 30, None) == E["E_WORKSPACE"]
        assert lib.stitch_grad_bind(h, 0x1001, 1 << 30, None) == E["E_WORKSPACE"]
    finally:
        lib.stitch_grad_destroy(h)
    bad = [m0, m0]
    assert _grad_create(bad, W, H, 3)[0] == E["E_MASK"]
    assert _grad_create(good, W, H, 0)[0] == E["E_LEVELS"]
    assert _grad_create(good, W, H, 6)[0] == E["E_LEVELS"]          # top level side below 3
    assert _grad_create(good, W, H, 2, fw=(0, 64))[0] == E["E_SHAPE"]
    assert lib.stitch_grad_create(None, None, None, W, H, 2, ctypes.byref(ctypes.c_void_p())) == E["E_NULL"]


def test_corner_parameterisation_matches_the_oracle_chain_rule():
    """Host FP64 code: DLT of the corners and the chain rule d loss/dM -> d loss/dq agree
    with the oracle's Jacobians; degenerate corners are rejected."""
    import oracle as o

    rng = np.random.default_rng(7)
    for _ in range(5):
        w, h = int(rng.integers(64, 1400)), int(rng.integers(48, 800))
        q = (o.corners(w, h) + rng.uniform(-0.2, 0.2, (4, 2)) * [w, h] + [900, 10]).ravel()
        Hq = P.corners_to_h(q, w, h)
        Ho = o.dlt_from_corners(q, w, h)
        assert np.allclose(Hq, Ho, rtol=1e-12, atol=1e-15)
        dm = rng.normal(size=9)
        want = o.dlt_jacobian(q, w, h).T @ (o.canvas_map_jacobian(Ho).T @ dm)
        got = P.map_grad_to_corners(q, w, h, dm)
        assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
    flat = np.array([0.0, 0, 10, 0, 20, 0, 30, 0])       # all four corners on one line
    with pytest.raises(P.StitchError) as e:
        P.corners_to_h(flat, 64, 48)
    assert e.value.status == E["E_HOMOGRAPHY"]


def test_binding_refuses_host_tensors_before_any_launch():
    """A host tensor's address given to a device call would make the kernel fault; the
    binding raises ValueError before anything reaches the library."""
    import torch
    t = torch.zeros((8, 8, 3), dtype=torch.uint8)
    with pytest.raises(ValueError):
        S.image_hwc(t)
    with pytest.raises(ValueError):
        S.image_chw(torch.zeros((3, 8, 8), dtype=torch.float32))
    pat = torch.zeros((32, 4), dtype=torch.int32)
    lorb = object.__new__(S.Lorb)
    with pytest.raises(ValueError):
        S.Lorb.run_raw(lorb, t, pat, 0)
    pro = object.__new__(S.Prosac)
    i32 = torch.zeros(8, dtype=torch.int32)
    with pytest.raises(ValueError):
        S.Prosac.run_raw(pro, i32, i32, i32, i32, i32, torch.zeros((4, 4), dtype=torch.float64), 0)
    mat = object.__new__(S.Matcher)
    with pytest.raises(ValueError):
        S.Matcher.run_raw(mat, i32, i32, i32, i32, 0)
    mset = object.__new__(S.MatcherSet)
    mset.n, mset.pairs = 1, (S.MatchPair * 1)()
    with pytest.raises(ValueError):
        S.MatcherSet.run_raw(mset, [(i32, i32, i32, i32)], 0)
    with pytest.raises(ValueError):
        S.MatcherSet.run_raw(mset, [], 0)
    pset = object.__new__(S.ProsacSet)
    pset.n, pset.pairs = 1, (S.ProsacPair * 1)()
    with pytest.raises(ValueError):
        S.ProsacSet.run_raw(pset, [(i32, i32, i32, i32, i32, torch.zeros((4, 4), dtype=torch.float64))], 0)
    # the validating forms check dtype, shape and device first
    mset.caps, mset.nd = [(8, 8)], 256
    d = torch.zeros((8, 16), dtype=torch.int32)
    with pytest.raises(ValueError, match="descriptors"):
        S.MatcherSet.run(mset, [(d, i32[:1], d, i32[:1])])
    pset.caps, pset.nhyp = [(8, 8)], 4
    with pytest.raises(ValueError, match="pts_a"):
        S.ProsacSet.run(pset, [(i32, i32, i32, i32, i32, torch.zeros((4, 4), dtype=torch.float64))])
    with pytest.raises(ValueError, match="uniforms"):
        S.ProsacSet.run(pset, [(i32, i32, i32, i32, i32, torch.zeros((3, 4), dtype=torch.float64))])


def test_frame_backward_validates_on_host():
    """The float-frame forward and its VJP: workspace size, NULLs, wrong dtypes, sizes and a
    misaligned or short workspace are refused before anything reaches the device."""
    lib = P.lib()
    args, keep = _plan_args()
    st, h = _create(*args)
    assert st == 0
    try:
        need = lib.stitch_frame_backward_workspace_bytes(h)
        W, H = 1040, 480
        assert need >= 13 * 8 * W * H and lib.stitch_frame_backward_workspace_bytes(None) == 0
        fake = 0x10000

        def img(w, hh, dtype=S.F32):
            return S.StitchImage(fake, w, hh, 3, dtype, S.CHW, 4 * w, 4 * w * hh)

        fr = (S.StitchImage * 2)(img(640, 480), img(640, 480))
        bad = (S.StitchImage * 2)(img(640, 480), img(639, 480))
        u8 = (S.StitchImage * 2)(img(640, 480), img(640, 480, S.U8))
        out = (S.StitchImage * 2)(img(640, 480), img(640, 480))
        dp = img(W, H)
        dh = (ctypes.c_double * 18)()

        def bwd(frames=fr, d_pano=ctypes.byref(dp), d_frames=out, ws=fake, nbytes=need, d_hinv=dh):
            return lib.stitch_frame_backward(h, frames, d_pano, None, d_frames, d_hinv, ws, nbytes, None)

        assert bwd(frames=None) == E["E_NULL"] and bwd(d_hinv=None) == E["E_NULL"]
        assert bwd(ws=None) == E["E_WORKSPACE"] and bwd(ws=fake + 8) == E["E_WORKSPACE"]
        assert bwd(nbytes=need - 1) == E["E_WORKSPACE"]
        assert bwd(frames=bad) == E["E_SHAPE"] and bwd(frames=u8) == E["E_SHAPE"]
        assert bwd(d_frames=bad) == E["E_SHAPE"]
        small = img(W - 1, H)
        assert bwd(d_pano=ctypes.byref(small)) == E["E_SHAPE"]
        r0 = img(W, H)
        assert lib.stitch_frame_forward_f32(h, fr, ctypes.byref(small), fake, need, None) == E["E_SHAPE"]
        assert lib.stitch_frame_forward_f32(h, bad, ctypes.byref(r0), fake, need, None) == E["E_SHAPE"]
        assert lib.stitch_frame_forward_f32(h, fr, ctypes.byref(r0), fake, need // 2, None) == E["E_WORKSPACE"]
    finally:
        lib.stitch_plan_destroy(h)
