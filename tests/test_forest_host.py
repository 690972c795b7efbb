"""Host forest (links, cuts, labels, roots, member collection) checked
against a naive adjacency-set model under random operations, including a
high-degree hub and long paths; built with address and undefined-behaviour
sanitizers (host code only)."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def binary():
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "forest_check")
    subprocess.check_call([
        "g++", "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=address,undefined",
        "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_2509_14433_amd", "csrc"),
        os.path.join(ROOT, "tests", "native", "forest_check.cpp"), "-o", exe])
    return exe


@pytest.mark.parametrize("V,steps,seed", [(8, 3000, 1), (60, 3000, 2), (200, 1500, 3),
                                          (2, 200, 4)])
def test_forest_matches_naive_model(binary, V, steps, seed):
    r = subprocess.run([binary, str(V), str(steps), str(seed)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.fixture(scope="module")
def contract_binary():
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "contract_check")
    subprocess.check_call([
        "g++", "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=address,undefined",
        "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_2509_14433_amd", "csrc"),
        os.path.join(ROOT, "tests", "native", "contract_check.cpp"), "-o", exe])
    return exe


@pytest.mark.parametrize("V,runs,seed,threads", [(8, 500, 1, 0), (60, 800, 2, 0), (200, 500, 3, 0),
                                                 (2, 100, 4, 0), (1000, 300, 5, 0),
                                                 (200, 500, 6, 4), (1000, 300, 7, 3)])
def test_contracted_walk_matches_one_by_one(contract_binary, V, runs, seed, threads):
    """The contracted walk of a run of flagged updates leaves the same
    forest edges, trees, dirty trees and link / cut counts as walking the
    run one update at a time; runs whose piece search is given too small a
    budget fall back without changing an edge.  With threads, the merged
    trees of every link_many are relabelled on a worker pool."""
    r = subprocess.run([contract_binary, str(V), str(runs), str(seed), str(threads)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
