"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point the public header declares, and rejects bad arguments
before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2509_04336_amd import inputs, nsmi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nsmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ns_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert {"ns_init", "ns_step", "ns_loglike_batch", "ns_evidence", "ns_free"} <= set(names)
    L = C.CDLL(nsmi.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_version_string():
    assert "gfx950" in nsmi.version()


def _spec_and_data():
    spec = inputs.tiny_event()
    return spec, np.zeros((spec.n_det, spec.n_bins), np.complex128)


@pytest.mark.parametrize("kw,needle", [
    (dict(n_live=2), "n_live"),
    (dict(num_delete=99), "num_delete"),
    (dict(num_delete=0), "num_delete"),
    (dict(walk0=6000), "walk0"),
    (dict(term_kind=3), "term_kind"),
    (dict(precision=7), "precision"),
])
def test_init_rejects_bad_config(kw, needle):
    spec, data = _spec_and_data()
    args = dict(n_live=100, num_delete=50, naccept=30, maxmcmc=5000, walk0=100)
    args.update(kw)
    with pytest.raises(nsmi.NSError) as ei:
        nsmi.Context([spec], [data], **args)
    assert ei.value.status == nsmi.NS_EINVAL
    assert needle in str(ei.value)


def test_init_rejects_nonfinite_data_and_bad_psd():
    spec, data = _spec_and_data()
    bad = data.copy()
    bad[0, 17] = np.nan
    with pytest.raises(nsmi.NSError) as ei:
        nsmi.Context([spec], [bad], n_live=10, num_delete=5, naccept=5, maxmcmc=10, walk0=5)
    assert ei.value.status == nsmi.NS_ENONFINITE
    import dataclasses
    psd = spec.psd.copy()
    psd[0, 3] = 0.0
    spec2 = dataclasses.replace(spec, psd=psd)
    with pytest.raises(nsmi.NSError) as ei:
        nsmi.Context([spec2], [data], n_live=10, num_delete=5, naccept=5, maxmcmc=10, walk0=5)
    assert ei.value.status == nsmi.NS_ENONFINITE


def test_init_rejects_bad_dimension():
    import dataclasses
    spec, data = _spec_and_data()
    spec2 = dataclasses.replace(spec, ndim=5)
    with pytest.raises(nsmi.NSError) as ei:
        nsmi.Context([spec2], [data], n_live=10, num_delete=5, naccept=5, maxmcmc=10, walk0=5)
    assert ei.value.status == nsmi.NS_EINVAL and "ndim" in str(ei.value)


def test_null_arguments():
    L = nsmi.lib()
    assert L.ns_init(None, None, None, 0) == nsmi.NS_EINVAL
    assert L.ns_step(None, 1, 1) == nsmi.NS_EINVAL
    assert L.ns_evidence(None, 0, None) == nsmi.NS_EINVAL
    L.ns_free(None)


def test_n_live_matching_helper():
    # Sec. 3.2.1: n_GPU = 2 ln 2 n_CPU at k = n/2; 1000 sequential -> ~1386
    assert nsmi.n_live_for_batch(1000) == 1386
    assert nsmi.n_live_for_batch(1000, 1e-6) == 1000


def test_binding_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures of the binding have the sizes and field offsets
    that a C compiler gives the header's structs."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"ns_event_desc": nsmi.EventDesc, "ns_config": nsmi.Config,
               "ns_timing_t": nsmi.Timing, "ns_evidence_t": nsmi.Evidence}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "nsmi.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            cname, field, val = line.split()
            got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
