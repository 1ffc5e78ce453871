"""Host-side checks of the C ABI: the library loads without a GPU, exports every
function include/vrm.h declares, and the Python binding's structures have the
header's layout (compared with a C program built against the header)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1508_06379_amd as vrm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vrm.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(vrm_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(vrm.LIB_PATH):
        pytest.skip("libvrm.so not built")
    return ctypes.CDLL(vrm.LIB_PATH)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(vrm.EXPORTS)


def test_status_strings(lib):
    lib.vrm_status_string.restype = ctypes.c_char_p
    assert lib.vrm_status_string(0) == b"ok"
    assert lib.vrm_status_string(-2) == b"capacity exceeded"
    assert b"non-finite" in lib.vrm_status_string(-5)


def test_create_rejects_bad_capacity(lib):
    h = ctypes.c_void_p()
    lib.vrm_last_error.restype = ctypes.c_char_p
    assert lib.vrm_create(ctypes.byref(h), 0, None, 0) == -1
    assert b"capacity" in lib.vrm_last_error()


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "vrm.h"
#define P(T, f) printf(#T "." #f " %zu\\n", offsetof(T, f));
int main(void) {
  printf("vrm_params %zu\\n", sizeof(vrm_params));
  printf("vrm_cloud %zu\\n", sizeof(vrm_cloud));
  printf("vrm_stencils %zu\\n", sizeof(vrm_stencils));
  printf("vrm_counters %zu\\n", sizeof(vrm_counters));
  printf("vrm_tuning %zu\\n", sizeof(vrm_tuning));
  P(vrm_params, q) P(vrm_params, deterministic) P(vrm_tuning, cert_rounds)
  printf("VRM_E_NONFINITE %d\\n", VRM_E_NONFINITE);
  printf("VRM_ST_WARM %d\\n", VRM_ST_WARM);
  P(vrm_cloud, capacity) P(vrm_stencils, full_f_dev)
  P(vrm_counters, n_small) P(vrm_counters, n_truncated) P(vrm_counters, n_grid_clamped) P(vrm_counters, pivots) P(vrm_counters, redistributions) P(vrm_counters, mis_rounds) P(vrm_counters, full_cols)
  P(vrm_counters, graph_replays) P(vrm_counters, cert_exact) P(vrm_tuning, infer_blocks) P(vrm_tuning, lp_small_lanes) P(vrm_tuning, lp_small_coop)
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)]).decode().splitlines())
    assert int(out["vrm_params"]) == ctypes.sizeof(vrm.vrm_params)
    assert int(out["vrm_cloud"]) == ctypes.sizeof(vrm.vrm_cloud)
    assert int(out["vrm_stencils"]) == ctypes.sizeof(vrm.vrm_stencils)
    assert int(out["vrm_counters"]) == ctypes.sizeof(vrm.vrm_counters)
    assert int(out["vrm_params.q"]) == vrm.vrm_params.q.offset
    assert int(out["vrm_params.deterministic"]) == vrm.vrm_params.deterministic.offset
    assert int(out["vrm_tuning.cert_rounds"]) == vrm.vrm_tuning.cert_rounds.offset
    assert int(out["VRM_E_NONFINITE"]) == vrm.E_NONFINITE
    assert int(out["VRM_ST_WARM"]) == vrm.ST_WARM
    assert int(out["vrm_cloud.capacity"]) == vrm.vrm_cloud.capacity.offset
    assert int(out["vrm_stencils.full_f_dev"]) == vrm.vrm_stencils.full_f_dev.offset
    assert int(out["vrm_counters.n_small"]) == vrm.vrm_counters.n_small.offset
    assert int(out["vrm_counters.n_truncated"]) == vrm.vrm_counters.n_truncated.offset
    assert int(out["vrm_counters.n_grid_clamped"]) == vrm.vrm_counters.n_grid_clamped.offset
    assert int(out["vrm_counters.pivots"]) == vrm.vrm_counters.pivots.offset
    assert int(out["vrm_counters.redistributions"]) == vrm.vrm_counters.redistributions.offset
    assert int(out["vrm_counters.mis_rounds"]) == vrm.vrm_counters.mis_rounds.offset
    assert int(out["vrm_counters.full_cols"]) == vrm.vrm_counters.full_cols.offset
    assert int(out["vrm_counters.graph_replays"]) == vrm.vrm_counters.graph_replays.offset
    assert int(out["vrm_counters.cert_exact"]) == vrm.vrm_counters.cert_exact.offset
    assert int(out["vrm_tuning"]) == ctypes.sizeof(vrm.vrm_tuning)
    assert int(out["vrm_tuning.infer_blocks"]) == vrm.vrm_tuning.infer_blocks.offset
    assert int(out["vrm_tuning.lp_small_lanes"]) == vrm.vrm_tuning.lp_small_lanes.offset
    assert int(out["vrm_tuning.lp_small_coop"]) == vrm.vrm_tuning.lp_small_coop.offset


def test_product_path_has_no_cpu_fallback():
    """The package never imports the oracle: it fails loudly without its HIP library."""
    src = open(os.path.join(ROOT, "paper_1508_06379_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("oracle", "", 0) or "import oracle" not in src
    assert "import oracle" not in src and "from oracle" not in src
