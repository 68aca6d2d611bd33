"""Host logic of bench.py's counted-traffic key (no GPU).

The counted HBM bytes of the fused operator kernel are reported only while
the source it compiles from is unchanged.  The key hashes nek_kernels.hpp up
to its gather-scatter section, so an edit to a kernel after that point keeps
the figure and an edit inside the operator's part drops it.
"""
import os
import shutil
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _copy_tree(tmp_path):
    for (rel, _), _digest in bench.COUNTER_TRAFFIC["sources"].items():
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, rel), dst)


def _append(path, before_marker, marker, extra):
    text = path.read_text()
    if before_marker:
        i = text.index(marker)
        text = text[:i] + extra + text[i:]
    else:
        text = text + extra
    path.write_text(text)


def test_region_key(tmp_path, monkeypatch):
    _copy_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (rel, marker), digest = next((k, v) for k, v in bench.COUNTER_TRAFFIC["sources"].items() if k[1])
    assert marker is not None
    before, reported = bench.operator_source_digest(rel, marker), bench.counter_traffic(5)
    assert (reported is not None) == (before == digest) or reported is None
    # an edit after the marker leaves the operator's digest and the figure as they were
    _append(tmp_path / rel, False, marker, "\n// another kernel\n")
    assert bench.operator_source_digest(rel, marker) == before
    assert bench.counter_traffic(5) == reported
    # an edit inside the operator's part changes it and drops the figure
    _append(tmp_path / rel, True, marker, "// operator edit\n")
    assert bench.operator_source_digest(rel, marker) != before
    assert bench.counter_traffic(5) is None
    assert bench.counter_traffic(4) is None


def test_missing_marker_never_matches(tmp_path, monkeypatch):
    _copy_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (rel, marker), _ = next((k, v) for k, v in bench.COUNTER_TRAFFIC["sources"].items() if k[1])
    path = tmp_path / rel
    path.write_text(path.read_text().replace(marker, "// renamed section"))
    assert bench.counter_traffic(5) is None
