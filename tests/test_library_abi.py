"""CPU checks of the C ABI: the library loads, exports every function that
include/truss.h declares, and its host-side logic (options, workspace sizing,
argument checks that fail before any device work) behaves as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "truss.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char|size_t)\s*\*?\s*(truss_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def T():
    import paper_1205_6693_amd as T
    return T


def test_header_lists_the_boundary():
    names = declared_functions()
    for f in ("truss_support", "truss_decompose", "truss_batch", "truss_workspace_size"):
        assert f in names


def test_library_exports_every_declared_symbol(T):
    lib = T.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_strerror(T):
    lib = T.load_library()
    assert lib.truss_version() == T.TRUSS_VERSION
    for code in range(0, -13, -1):
        assert lib.truss_strerror(code)
    assert lib.truss_strerror(-99) == b"unknown error"


def test_struct_layouts_match_header(T):
    # sizes of the ABI structs: graph 48 B, options 64 B, stats 208 B (options
    # keep their size: batch_block and batch_ilp took two reserved words)
    assert ctypes.sizeof(T._Graph) == 48
    assert ctypes.sizeof(T.Options) == 64
    assert ctypes.sizeof(T.Stats) == 208


def _graph(T, n, m, fmt=0):
    g = T._Graph()
    g.n, g.m, g.fmt = n, m, fmt
    g.src = g.dst = g.row_ptr = g.col = 4096  # never dereferenced by the size query
    return g


def test_workspace_size_is_host_only_and_grows(T):
    lib = T.load_library()
    sizes = []
    for m in (0, 10, 1000, 100000):
        b = ctypes.c_size_t(0)
        assert lib.truss_workspace_size(ctypes.byref(_graph(T, 100, m)), None, ctypes.byref(b)) == 0
        sizes.append(b.value)
    assert sizes == sorted(sizes) and sizes[-1] > 100000 * 40
    b = ctypes.c_size_t(0)
    assert lib.truss_workspace_size(ctypes.byref(_graph(T, 100, 1000, fmt=1)), None, ctypes.byref(b)) == 0


def test_argument_errors_before_device_work(T):
    lib = T.load_library()
    b = ctypes.c_size_t(0)
    assert lib.truss_workspace_size(None, None, ctypes.byref(b)) == T.E_INVAL
    assert lib.truss_workspace_size(ctypes.byref(_graph(T, -1, 5)), None, ctypes.byref(b)) == T.E_INVAL
    assert lib.truss_workspace_size(ctypes.byref(_graph(T, 5, 1 << 31)), None, ctypes.byref(b)) == T.E_TOOBIG
    assert lib.truss_workspace_size(ctypes.byref(_graph(T, 5, 5, fmt=7)), None, ctypes.byref(b)) == T.E_INVAL
    o = T.Options()
    lib.truss_default_options(ctypes.byref(o))
    assert o.version == T.TRUSS_VERSION
    o.version = 1
    assert lib.truss_workspace_size(ctypes.byref(_graph(T, 5, 5)), ctypes.byref(o), ctypes.byref(b)) == T.E_INVAL
    o.version = T.TRUSS_VERSION
    o.peel_mode = 9
    assert lib.truss_workspace_size(ctypes.byref(_graph(T, 5, 5)), ctypes.byref(o), ctypes.byref(b)) == T.E_INVAL
    o.peel_mode = 0
    for shape in (T.SHAPE_AUTO, T.SHAPE_NARROW, T.SHAPE_WIDE):
        o.peel_shape = shape
        assert lib.truss_workspace_size(ctypes.byref(_graph(T, 5, 5)), ctypes.byref(o), ctypes.byref(b)) == T.OK
    o.peel_shape = 3
    assert lib.truss_workspace_size(ctypes.byref(_graph(T, 5, 5)), ctypes.byref(o), ctypes.byref(b)) == T.E_INVAL
    o.peel_shape = 0
    # decompose with NULL output or too small workspace fails on the host
    g = _graph(T, 5, 5)
    assert lib.truss_decompose(ctypes.byref(g), None, None, None, None, 0, None) == T.E_INVAL
    out = ctypes.c_void_p(4096)
    assert lib.truss_decompose(ctypes.byref(g), out, None, None, None, 0, None) == T.E_WORKSPACE
    assert b"workspace" in lib.truss_last_error()


def test_batch_workspace_covers_slots_and_big_graphs(T):
    import numpy as np
    lib = T.load_library()
    # three small graphs: one scratch slot each, sized for the largest (180 edges)
    vo = np.array([0, 10, 30, 31], np.int64)
    eo = np.array([0, 20, 200, 200], np.int64)
    small = T.truss_batch_workspace_size(vo, eo)
    assert small >= 3 * 48 * 180
    # one more graph above the persistent kernel's limit (2^21 edges) adds the
    # device-wide path's workspace for it
    big_m = (1 << 21) + 5
    vo2 = np.append(vo, vo[-1] + 1_000_000)
    eo2 = np.append(eo, eo[-1] + big_m)
    with_big = T.truss_batch_workspace_size(vo2, eo2)
    b = ctypes.c_size_t(0)
    assert lib.truss_workspace_size(ctypes.byref(_graph(T, 1_000_000, big_m)), None, ctypes.byref(b)) == 0
    assert with_big >= small + b.value
    # bad offsets and bad batch shapes are rejected on the host
    with pytest.raises(T.TrussError):
        T.truss_batch_workspace_size(np.array([0, 5, 3], np.int64), np.array([0, 1, 2], np.int64))
    with pytest.raises(T.TrussError):
        T.truss_batch_workspace_size(vo, eo, T.make_options(batch_block=300))


def test_trace_layout_and_network_sizes(T):
    # trace: 2 ints, 3 pointers, 4 actions, 4 x 6 features, 4 times
    assert ctypes.sizeof(T.Trace) == 8 + 24 + 16 + 96 + 16
    lib = T.load_library()
    assert T.mlp_param_count(8, 32, 4) == 32 * 8 + 32 + 4 * 32 + 4
    assert lib.truss_mlp_param_count(0, 4, 4) == T.E_INVAL
    assert lib.truss_mlp_param_count(17, 4, 4) == T.E_INVAL
    assert lib.truss_mlp_param_count(8, 65, 4) == T.E_INVAL
    assert lib.truss_mlp_param_count(8, 4, 9) == T.E_INVAL
    # a model part: header, normalisation, parameters
    assert T.sched_part_floats(0, 32) == 4 + 2 * 8 + T.mlp_param_count(8, 32, 4)
    assert T.sched_part_floats(1, 16) == 4 + 2 * 6 + T.mlp_param_count(6, 16, 3)
    assert lib.truss_sched_model_floats(32) == T.sched_part_floats(0, 32) + T.sched_part_floats(1, 32)
    assert lib.truss_sched_part_floats(2, 32) == T.E_INVAL
    b = ctypes.c_size_t(0)
    assert lib.truss_mlp_workspace_size(8, 32, 4, 1000, ctypes.byref(b)) == 0 and b.value > 1000 * 32 * 4
    assert lib.truss_mlp_workspace_size(8, 32, 4, 0, ctypes.byref(b)) == T.E_INVAL
    assert lib.truss_sched_train_workspace_size(0, 32, 100, ctypes.byref(b)) == 0
    # host-side argument checks of the network entry points
    assert lib.truss_mlp_forward(None, 8, 32, 4, None, 10, None, None, 0, None) == T.E_INVAL
    p = ctypes.c_void_p(4096)
    assert lib.truss_mlp_forward(p, 8, 32, 4, p, 10, p, None, 0, None) == T.E_WORKSPACE
    assert lib.truss_mlp_train(p, p, p, 8, 32, 4, p, p, p, 10, 5, 0, ctypes.c_float(0.0), None, None, 0,
                               None) == T.E_INVAL
    tr = T.Trace()
    g = _graph(T, 5, 5)
    assert lib.truss_decompose_traced(ctypes.byref(g), p, None, None, None, None, 0, None) == T.E_INVAL
    tr.level_cap = 4
    assert lib.truss_decompose_traced(ctypes.byref(g), p, None, None, ctypes.byref(tr), None, 0,
                                      None) == T.E_WORKSPACE


def test_core_and_cohesion_sizes_and_errors(T):
    lib = T.load_library()
    assert ctypes.sizeof(T.CohesionStats) == 64
    b = ctypes.c_size_t(0)
    assert lib.truss_core_workspace_size(ctypes.byref(_graph(T, 1000, 5000)), ctypes.byref(b)) == 0
    core_bytes = b.value
    assert core_bytes >= 1000 * 12
    assert lib.truss_cohesion_workspace_size(ctypes.byref(_graph(T, 1000, 5000)), ctypes.byref(b)) == 0
    assert b.value > core_bytes
    assert lib.truss_core_workspace_size(None, ctypes.byref(b)) == T.E_INVAL
    assert lib.truss_cohesion_workspace_size(ctypes.byref(_graph(T, -1, 5)), ctypes.byref(b)) == T.E_INVAL
    # too small a workspace and missing outputs fail before any device call
    g = _graph(T, 1000, 5000)
    cmax = ctypes.c_int32(0)
    assert lib.truss_core_numbers(ctypes.byref(g), None, ctypes.byref(cmax), None, 0, None) == T.E_INVAL
    assert lib.truss_core_numbers(ctypes.byref(g), 4096, ctypes.byref(cmax), 4096, 16, None) == T.E_WORKSPACE
    st = T.CohesionStats()
    assert lib.truss_cohesion(ctypes.byref(g), None, None, 4096, 1 << 40, None) == T.E_INVAL
    assert lib.truss_cohesion(ctypes.byref(g), None, ctypes.byref(st), 4096, 16, None) == T.E_WORKSPACE


def test_bottomup_sizes_and_errors(T):
    lib = T.load_library()
    assert ctypes.sizeof(T.BottomUpStats) == 128
    b = ctypes.c_size_t(0)
    assert lib.truss_bottomup_workspace_size(0, ctypes.byref(b)) == T.E_INVAL
    assert lib.truss_bottomup_workspace_size(1000, ctypes.byref(b)) == 0 and b.value > 1000 * 17
    small = b.value
    assert lib.truss_bottomup_workspace_size(100000, ctypes.byref(b)) == 0 and b.value > small
    import numpy as np
    s = np.array([0, 2], np.int32)
    d = np.array([1, 2], np.int32)
    out = np.zeros(2, np.int32)
    st = T.BottomUpStats()
    # too small a workspace, then a self-loop found on the host before any device work
    assert lib.truss_bottomup(4, 2, s.ctypes.data, d.ctypes.data, None, 10, out.ctypes.data, None, None,
                              ctypes.byref(st), 4096, 16, None) == T.E_WORKSPACE
    assert lib.truss_bottomup(4, 2, s.ctypes.data, d.ctypes.data, None, 10, out.ctypes.data, None, None,
                              ctypes.byref(st), 4096, 1 << 40, None) == T.E_SELFLOOP
    d2 = np.array([1, 4], np.int32)
    assert lib.truss_bottomup(4, 2, s.ctypes.data, d2.ctypes.data, None, 10, out.ctypes.data, None, None,
                              ctypes.byref(st), 4096, 1 << 40, None) == T.E_RANGE


def test_binding_refuses_what_the_library_cannot_check(T):
    """The library dereferences the binding's tensors on the device: host
    tensors, wrong sizes and wrong lengths are refused in Python first."""
    import numpy as np
    import torch
    s = torch.tensor([0, 1], dtype=torch.int32)
    d = torch.tensor([1, 2], dtype=torch.int32)
    with pytest.raises(ValueError, match="device memory"):
        T.Graph.from_edges(3, s, d)
    with pytest.raises(ValueError):
        T.Graph.from_edges(3, s, d[:1])
    with pytest.raises(ValueError, match="n . 1 offsets"):
        T.Graph.from_csr(3, torch.tensor([0, 1, 2], dtype=torch.int64), torch.tensor([1, 0], dtype=torch.int32))
    with pytest.raises(ValueError, match="device memory"):
        T.Graph.from_csr(2, torch.tensor([0, 1, 2], dtype=torch.int64), torch.tensor([1, 0], dtype=torch.int32))
    with pytest.raises(ValueError, match="model"):
        T.make_options(model=torch.zeros(8))
    with pytest.raises(ValueError, match="edge_off"):  # 3 edges named, 2 given
        T.truss_batch([0, 3], [0, 3], s, d)
    with pytest.raises(ValueError, match="offset per graph"):
        T.truss_batch([0, 3], [0, 1, 2], s, d)
    with pytest.raises(ValueError, match="device memory"):
        T.truss_batch([0, 3], [0, 2], s, d)
    sn, dn = np.array([0, 1], np.int32), np.array([1, 2], np.int32)
    with pytest.raises(ValueError, match="one part id per vertex"):
        T.truss_bottomup(3, sn, dn, 10, first_part=np.zeros(2, np.int32))
    with pytest.raises(ValueError):
        T.truss_bottomup(3, sn, dn[:1], 10)


def test_bottomup_host_allocation_failure_is_a_status():
    """The bottom-up entry holds host memory in proportion to the graph; when
    it runs out the call returns TRUSS_E_NOMEM instead of ending the process.
    A child process caps its address space 1 GiB above what it uses after
    loading the library and asks for an adjacency of 400M vertices (3.2 GB of
    offsets); the edges are validated and the adjacency built before any
    device work, so no GPU is needed."""
    import subprocess
    import sys
    code = "\n".join([
        "import ctypes, resource, sys",
        "sys.path.insert(0, %r)" % ROOT,
        "import numpy as np",
        "import paper_1205_6693_amd as T",
        "lib = T.load_library()",
        "s, d, out = np.array([0], np.int32), np.array([1], np.int32), np.zeros(1, np.int32)",
        "st = T.BottomUpStats()",
        "vm = [int(l.split()[1]) for l in open('/proc/self/status') if l.startswith('VmSize')][0] * 1024",
        "resource.setrlimit(resource.RLIMIT_AS, (vm + (1 << 30), vm + (1 << 30)))",
        "rc = lib.truss_bottomup(400000000, 1, s.ctypes.data, d.ctypes.data, None, 10, out.ctypes.data, None,",
        "                        None, ctypes.byref(st), 4096, 1 << 40, None)",
        "print('rc', rc, lib.truss_last_error().decode())",
    ])
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "rc -9 host memory allocation failed" in r.stdout


def test_cohen_workspace(T):
    lib = T.load_library()
    b = ctypes.c_size_t(0)
    assert lib.truss_cohen_workspace_size(ctypes.byref(_graph(T, 1000, 5000)), ctypes.byref(b)) == 0
    assert b.value > 5000 * 16
    assert lib.truss_cohen_workspace_size(None, ctypes.byref(b)) == T.E_INVAL
    g = _graph(T, 1000, 5000)
    assert lib.truss_cohen(ctypes.byref(g), 4096, None, 4096, 16, None) == T.E_WORKSPACE


def test_missing_library_fails_loudly(tmp_path):
    """No CPU fallback: without the built library the binding raises."""
    import subprocess
    import sys
    code = ("import paper_1205_6693_amd as T; T.LIB_PATH = %r\n"
            "try:\n    T.load_library()\nexcept ImportError as e:\n    print('raised', e)\n" % str(tmp_path / "none.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert "raised" in r.stdout and "not built" in r.stdout, r.stdout + r.stderr


def test_noalloc_refuses_oversized_graph_without_device_work(T):
    """truss_decompose_noalloc checks the graph's scratch need against its
    fixed array before touching a device (so this runs without a GPU)."""
    lib = T.load_library()
    st = T.Stats()
    rc = lib.truss_decompose_noalloc(ctypes.byref(_graph(T, 1 << 20, 4 << 20)), ctypes.c_void_p(4096), None,
                                     ctypes.byref(st), None)
    assert rc == T.E_WORKSPACE
    assert b"fixed array" in lib.truss_last_error()
    assert lib.truss_decompose_noalloc(None, None, None, None, None) == T.E_INVAL
