"""C-ABI checks that need no GPU: libcox.so loads, exports every entry point
that include/cox.h declares, and rejects bad arguments on the host before
launching anything."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cox.h")
LIB = os.path.join(ROOT, "paper_2112_10034_amd", "libcox.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cox_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def cox():
    if not os.path.exists(LIB):
        import __graft_entry__

        __graft_entry__.build()
    from paper_2112_10034_amd import cox as binding

    return binding


def test_header_declares_the_hot_path():
    names = declared_functions()
    for must in ["cox_warp_reduce", "cox_warp_scan", "cox_ballot_compact", "cox_tile_sort",
                 "cox_tile_reduce", "cox_warp_masked", "cox_warp_dot", "cox_warp_shfl",
                 "cox_warp_vote", "cox_tile_vote", "cox_warp_reduce_blocks_i32"]:
        assert must in names


def test_library_exports_every_declared_symbol(cox):
    lib = C.CDLL(cox.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared entry points
    assert set(cox.exported_symbols()) <= set(declared_functions())


def test_host_only_queries(cox):
    L = cox.lib()
    assert L.cox_version() >= 100
    assert L.cox_status_string(0) == b"ok"
    assert b"aligned" in L.cox_status_string(3)
    k, W, G = cox.default_cfg(cox.OP_SCAN)
    assert k in (1, 2, 4, 8, 16, 32) and W in (1, 2, 4, 8, 16, 32) and G == 0
    n = 1 << 20
    S = 32 * W * k
    # status words one per 128-byte line
    assert L.cox_workspace_bytes(cox.OP_SCAN, cox.I32, n, 0, None) == 256 + 128 * (-(-n // S) + 1)
    assert L.cox_workspace_bytes(cox.OP_COMPACT, cox.I32, n, 0, None) == 256 + 128 * (-(-n // S) + 1)
    assert L.cox_workspace_bytes(cox.OP_SCAN, cox.I32, -1, 0, None) == 0
    bad = cox.make_cfg(3, 8)
    assert L.cox_workspace_bytes(cox.OP_REDUCE, cox.F32, n, 0, C.byref(bad)) == 0


def test_invalid_arguments_rejected_before_launch(cox):
    L = cox.lib()
    # negative sizes, bad widths / tiles / ops, missing workspace: no launch happens
    assert L.cox_warp_shfl(None, None, -32, 0, 0, None, 32, None, None) == 1
    assert L.cox_warp_shfl(None, None, 33, 0, 0, None, 32, None, None) == 1
    assert L.cox_warp_shfl(None, None, 32, 0, 0, None, 3, None, None) == 1
    assert L.cox_warp_shfl(None, None, 32, 2, 32, None, 32, None, None) == 1
    assert L.cox_warp_shfl(None, None, 32, 7, 0, None, 32, None, None) == 1
    assert L.cox_tile_reduce(None, 64, 3, None, None) == 1
    assert L.cox_tile_sort(None, None, 64, 16, None, None) == 1
    assert L.cox_warp_masked(None, 33, 512, None, None, None) == 1
    assert L.cox_warp_masked(None, 64, 2000, None, None, None) == 1
    assert L.cox_warp_reduce(None, cox.I32, 10, cox.TWOSUM, None, None, C.c_void_p(8), None, 0, None) == 2
    assert L.cox_warp_dot(None, None, cox.I32, 10, 0, None, None, C.c_void_p(8), None, 0, None) == 2
    assert L.cox_warp_scan(None, None, -1, None, None, 0, None) == 1
    # misaligned data pointer
    assert L.cox_warp_scan(C.c_void_p(4), C.c_void_p(16), 100, None, C.c_void_p(256), 10**6, None) == 3
    # workspace too small
    assert L.cox_warp_scan(C.c_void_p(16), C.c_void_p(16), 100, None, C.c_void_p(256), 8, None) == 5
    bad = cox.make_cfg(3, 8)
    assert L.cox_warp_scan(C.c_void_p(16), C.c_void_p(16), 100, C.byref(bad), None, 0, None) == 1


def _up256(v):
    return (v + 255) // 256 * 256


def test_workspace_sizes_of_the_widened_operations(cox):
    L = cox.lib()
    assert cox.default_cfg(cox.OP_CG, cox.F32) == (4, 32, 0)
    for n in (0, 1, 1000, 1 << 20):
        S = 32 * 32 * 4
        nch = -(-n // S)
        want = 256 + 2048 + 256 + 4 * _up256(4 * n) + 2 * _up256(8 * nch)
        assert L.cox_workspace_bytes(cox.OP_CG, cox.F32, n, 0, None) == want
    for G in (1, 256):
        assert L.cox_workspace_bytes(cox.OP_GRID_EXCHANGE, cox.U32, G, 0, None) == 256 + 2048 + 4096 * G
    for H, W in ((1, 1), (65, 1025), (8192, 8192)):
        nb, ns = -(-H // 64), -(-W // 1024)
        want = 256 + _up256(4 * nb * W) + _up256(4 * ns * H) + _up256(4 * nb * ns)
        assert L.cox_workspace_bytes(cox.OP_INTEGRAL_IMAGE, cox.U32, H, W, None) == want
    assert L.cox_workspace_bytes(cox.OP_INTEGRAL_IMAGE, cox.U32, 4, -1, None) == 0


def test_widened_entry_points_reject_bad_arguments_before_launch(cox):
    L = cox.lib()
    P = C.c_void_p
    # tile sort: tiles that are not powers of two in [32, 1024], unsupported keys per lane
    assert L.cox_tile_sort(None, None, 64, 48, None, None) == 1
    assert L.cox_tile_sort(None, None, 64, 2048, None, None) == 1
    assert L.cox_tile_sort(None, None, 64, 64, C.byref(cox.make_cfg(2, 0)), None) == 6
    assert L.cox_tile_sort(None, None, 0, 1024, None, None) == 0
    # key-value sort: size, tile, keys per lane, aliasing, alignment
    assert L.cox_tile_sort_kv(None, None, None, None, -1, 32, None, None) == 1
    assert L.cox_tile_sort_kv(None, None, None, None, 64, 64, None, None) == 1
    assert L.cox_tile_sort_kv(None, None, None, None, 64, 32, C.byref(cox.make_cfg(16, 0)), None) == 6
    assert L.cox_tile_sort_kv(P(16), P(256), P(32), P(256), 64, 32, None, None) == 1
    assert L.cox_tile_sort_kv(P(16), P(256), P(36), P(512), 64, 32, None, None) == 3
    # integral image: negative shape, empty image, missing buffers, small workspace
    assert L.cox_integral_image(None, -1, 5, None, None, 0, None) == 1
    assert L.cox_integral_image(None, 0, 5, None, None, 0, None) == 0
    assert L.cox_integral_image(None, 5, 5, None, None, 0, None) == 1
    assert L.cox_integral_image(P(16), 5, 5, P(16), P(256), 16, None) == 5
    # grid exchange and its failure check
    assert L.cox_grid_exchange(0, 1, P(16), None, 0, None) == 1
    assert L.cox_grid_exchange(4, -1, P(16), None, 0, None) == 1
    assert L.cox_grid_exchange_absent(4, 1, 4, 10, P(16), None, 0, None) == 1
    assert L.cox_grid_exchange_absent(4, 1, 0, 0, P(16), None, 0, None) == 1
    # conjugate gradient: sizes, missing result, schedules, workspace
    cg = L.cox_cg_solve
    args = (P(16), P(16), P(16), 100, 300, P(16), P(16), 5, C.c_double(0.0), P(16), None)
    assert cg(P(16), P(16), P(16), -1, 0, P(16), P(16), 5, C.c_double(0.0), P(16), None, None, None, 0, None) == 1
    assert cg(*args[:9], None, None, None, None, 0, None) == 1
    assert cg(*args, C.byref(cox.make_cfg(4, 4)), P(256), 1 << 30, None) == 6
    assert cg(*args, C.byref(cox.make_cfg(3, 32)), P(256), 1 << 30, None) == 1
    assert cg(*args, None, P(256), 64, None) == 5
    assert L.cox_cg_solve_per_phase(*args, None, P(256), 64, None) == 5


def _declarations_with_context():
    """(name, own comment, section banner) for every cox_ function declared
    in include/cox.h, in order."""
    import re

    src = open(os.path.join(ROOT, "include", "cox.h")).read()
    banner, last, out = "", "", []
    for m in re.finditer(r"/\*.*?\*/|^[A-Za-z_][\w \*]*?\b(cox_\w+)\s*\(", src, re.S | re.M):
        t = m.group(0)
        if t.startswith("/*"):
            t = re.sub(r"\n\s*\*(?!/)", " ", t)
            if t.startswith("/* ----"):
                banner, last = t, ""
            else:
                last = t
        else:
            out.append((m.group(1), last, banner))
    return out


def test_every_declaration_cites_its_passage():
    """Every entry point's comment (or the banner of its section) cites the
    paper's section, table or code listing it follows, or says that no
    passage of the paper defines it (plumbing and measurement kernels)."""
    import re

    cite = re.compile(r"(Sec\.|[Ss]ection|Table|Code|Appendix|Algorithm)\s*~?\d")
    decls = _declarations_with_context()
    assert len(decls) >= 30
    missing = []
    for name, own, banner in decls:
        ctx = own + banner
        flat = " ".join(ctx.split())
        # the allocation-free variant names the callers it serves in place of a passage
        if not (cite.search(ctx) or "no passage of the paper" in flat or "callers that cannot allocate" in flat):
            missing.append(name)
    assert not missing, f"declarations without a cited passage: {missing}"
    # the compute entry points cite a passage of their own or of their section
    compute = [d for d in decls if not re.search(r"no passage of the paper", " ".join((d[1] + d[2]).split()))]
    assert {"cox_warp_scan", "cox_ballot_compact", "cox_tile_sort", "cox_tile_sort_kv",
            "cox_warp_masked", "cox_warp_reduce", "cox_warp_dot"} <= {d[0] for d in compute}
    for name in ("cox_warp_scan", "cox_ballot_compact", "cox_tile_sort", "cox_tile_sort_kv", "cox_warp_masked"):
        own = next(d[1] for d in decls if d[0] == name)
        assert cite.search(own), f"{name} has no citation of its own"


def test_noalloc_scan_rejects_sizes_beyond_its_scratch(cox):
    """The allocation-free scan refuses a call whose look-back words would not
    fit its fixed device scratch, before touching the device."""
    L = cox.lib()
    cap = 1 << 20
    fake = C.c_void_p(1 << 12)  # never dereferenced: every check below fails on the host
    small = cox.make_cfg(1, 1)  # 32 elements per chunk
    n_over = ((cap - 256) // 8) * 32  # one chunk more than the scratch holds
    assert 256 + 8 * (n_over // 32 + 1) > cap >= 256 + 8 * (n_over // 32)  # packed 8-byte status words
    assert L.cox_warp_scan_noalloc(fake, fake, n_over, C.byref(small), None, None) == 5
    assert L.cox_warp_scan_noalloc(fake, fake, -1, None, None, None) == 1
    assert L.cox_warp_scan_noalloc(None, fake, 64, None, None, None) == 1
    assert L.cox_warp_scan_noalloc(C.c_void_p((1 << 12) + 4), fake, 64, None, None, None) == 3
    bad = cox.make_cfg(3, 8)
    assert L.cox_warp_scan_noalloc(fake, fake, 64, C.byref(bad), None, None) != 0


def test_tile_vote_rejects_bad_arguments(cox):
    """Checked on the host before anything is launched."""
    L = cox.lib()
    fake = C.c_void_p(1 << 12)
    for tile in (0, 3, 64):
        assert L.cox_tile_vote(fake, 64, tile, fake, fake, None) == 1
    assert L.cox_tile_vote(fake, 33, 4, fake, fake, None) == 1
    assert L.cox_tile_vote(fake, -32, 4, fake, fake, None) == 1
    assert L.cox_tile_vote(None, 64, 4, fake, fake, None) == 1
    assert L.cox_tile_vote(None, 0, 4, None, None, None) == 0
