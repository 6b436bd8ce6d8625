"""No C++ exception crosses the C ABI.

1. The guard (csrc/abi_guard.hpp) compiled with g++: entry points written as
   function-try-blocks with its handler turn std::bad_alloc into
   MXL_ERR_OUT_OF_MEMORY and every other exception into MXL_ERR_INTERNAL,
   record a message naming the entry point, and recording an error never
   allocates (long messages are truncated into the fixed buffer).
2. Every entry point the header declares is defined in csrc/ as such a
   function-try-block (the two that return strings only return a pointer).
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_16852_amd", "csrc")
HANDLER = re.compile(r"^\}\s*catch\s*\(\.\.\.\)\s*\{\s*return\s+mxl::abi_exception\(__func__\);\s*\}",
                     re.S)

GUARD_TEST = r"""
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>
#include "abi_guard.hpp"

static mxl_status ok_body(int *out) try {
    *out = 7;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

static mxl_status throws_bad_alloc() try {
    throw std::bad_alloc();
} catch (...) {
    return mxl::abi_exception(__func__);
}

static mxl_status huge_vector(size_t n) try {
    std::vector<double> v(n);           // too large: std::bad_alloc or std::length_error
    v[0] = 1.0;
    return MXL_OK;
} catch (...) {
    return mxl::abi_exception(__func__);
}

static mxl_status throws_runtime() try {
    throw std::runtime_error("planted");
} catch (...) {
    return mxl::abi_exception(__func__);
}

static mxl_status throws_int() try {
    throw 42;
} catch (...) {
    return mxl::abi_exception(__func__);
}

int main() {
    int v = 0;
    const int st = (int)ok_body(&v);
    std::printf("ok %d %d\n", st, v);
    std::printf("bad_alloc %d %s\n", (int)throws_bad_alloc(), mxl::last_error());
    std::printf("huge %d %s\n", (int)huge_vector((size_t)1 << 61), mxl::last_error());
    std::printf("runtime %d %s\n", (int)throws_runtime(), mxl::last_error());
    std::printf("int %d %s\n", (int)throws_int(), mxl::last_error());
    std::string longmsg(5000, 'x');
    mxl::record_error(MXL_ERR_DEVICE, longmsg.c_str());
    std::printf("trunc %zu\n", std::strlen(mxl::last_error()));
    return 0;
}
"""


@pytest.fixture(scope="module")
def guard_run(tmp_path_factory):
    d = tmp_path_factory.mktemp("guard")
    src = d / "guard_test.cpp"
    src.write_text(GUARD_TEST)
    exe = d / "guard_test"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {ln.split(" ", 1)[0]: ln.split(" ", 1)[1] for ln in out.strip().splitlines()}


def _status(line):
    return int(line.split(" ", 1)[0])


def test_guard_passes_results_through(guard_run):
    assert guard_run["ok"] == "0 7"


def test_guard_maps_bad_alloc_to_out_of_memory(guard_run):
    assert _status(guard_run["bad_alloc"]) == 7
    assert "throws_bad_alloc: host memory allocation failed" in guard_run["bad_alloc"]


def test_guard_maps_oversized_allocation(guard_run):
    # libstdc++ reports an impossible vector size as length_error (INTERNAL) or
    # bad_alloc (OUT_OF_MEMORY); either way a status, not a termination
    assert _status(guard_run["huge"]) in (7, 10)
    assert "huge_vector:" in guard_run["huge"]


def test_guard_maps_other_exceptions_to_internal(guard_run):
    assert _status(guard_run["runtime"]) == 10
    assert "throws_runtime: internal error: planted" in guard_run["runtime"]
    assert _status(guard_run["int"]) == 10
    assert "unknown exception" in guard_run["int"]


def test_error_text_is_truncated_not_reallocated(guard_run):
    assert guard_run["trunc"] == "511"


def _declared():
    txt = open(os.path.join(ROOT, "include", "mxl.h")).read()
    status = set(re.findall(r"^mxl_status\s+(mxl_\w+)\s*\(", txt, re.M))
    strings = set(re.findall(r"^const char \*\s*(mxl_\w+)\s*\(", txt, re.M))
    return status, strings


def _definitions():
    """name -> source text from the end of the parameter list to the end of
    the definition's handler, for every definition of an mxl_* function."""
    defs = {}
    for fn in sorted(os.listdir(CSRC)):
        if not fn.endswith(".hip"):
            continue
        s = open(os.path.join(CSRC, fn)).read()
        for m in re.finditer(r'^(?:extern "C" )?(?:mxl_status|const char \*)\s*(mxl_\w+)\(', s, re.M):
            j, depth = m.end() - 1, 0
            while True:
                depth += {"(": 1, ")": -1}.get(s[j], 0)
                if depth == 0:
                    break
                j += 1
            rest = s[j + 1:]
            if rest.lstrip().startswith(";"):
                continue
            assert m.group(1) not in defs, f"{m.group(1)} defined twice"
            defs[m.group(1)] = (fn, rest)
    return defs


def test_every_entry_point_is_guarded():
    status, strings = _declared()
    defs = _definitions()
    assert status | strings == set(defs), sorted((status | strings) ^ set(defs))
    unguarded = []
    for name in sorted(status):
        fn, rest = defs[name]
        if not rest.lstrip().startswith("try {"):
            unguarded.append(f"{fn}:{name} (no function-try-block)")
            continue
        # the body's closing brace is followed by the guard's handler
        body = rest.lstrip()[len("try "):]
        depth, k = 0, 0
        while True:
            depth += {"{": 1, "}": -1}.get(body[k], 0)
            if depth == 0:
                break
            k += 1
        if not HANDLER.match(body[k:]):
            unguarded.append(f"{fn}:{name} (handler is not mxl::abi_exception)")
    assert not unguarded, unguarded


def test_string_entry_points_cannot_throw():
    _, strings = _declared()
    defs = _definitions()
    for name in strings:
        body = defs[name][1].strip()
        assert re.match(r'^\{\s*return\s+(mxl::last_error\(\)|"[^"]*");\s*\}', body), (name, body[:80])
