"""The set-up's sparse products on the device (expansion, stable radix sort
by row and column, in-order sums) give the host products' hierarchy bit for
bit: the hierarchy files that mdp_save writes are byte-identical, and so are
the solves.  With MDP_DEVICE_PRODUCT_TERMS=1 every product goes to the
device, including small ones with empty rows and cancelling terms."""

import os

import pytest
import torch

import synth
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa, tpfa_flux

from gpu_common import dev, say

pytestmark = pytest.mark.gpu


def _file(tmp_path, A, part, flags, name, labels=None):
    h = L.mdp_setup(A, part, L.mdp_options_default(flags=flags), labels=labels)
    path = tmp_path / name
    try:
        L.mdp_save(h, str(path))
    finally:
        L.mdp_destroy(h)
    return path.read_bytes()


def _same_hierarchy(tmp_path, A, part, labels=None):
    dev_bytes = _file(tmp_path, A, part, 0, "dev.mdph", labels)
    host_bytes = _file(tmp_path, A, part, L.MDP_HOST_PRODUCTS, "host.mdph", labels)
    assert len(dev_bytes) == len(host_bytes)
    assert dev_bytes == host_bytes


CASES = {
    "tiny_2d": lambda: tpfa.assemble(synth.tiny_2d(12)),
    "tiny_3d": lambda: tpfa.assemble(synth.tiny_3d(8)),
    "four lines 32 (uniform host)": lambda: tpfa.assemble(synth.grid_2d_four_lines(32)),
    "random_2d seed 3": lambda: tpfa.assemble(synth.random_2d(3, n_range=(64, 128))),
    "regular_3d 24": lambda: tpfa.assemble(synth.regular_3d(n=24, k_par=1e-4, kappa=1e4, seed=2)),
    "flux 3d 12": lambda: tpfa_flux.assemble_flux(synth.regular_3d(n=12, seed=1))[:3],
}


@pytest.mark.parametrize("name", list(CASES))
def test_every_product_on_the_device_gives_the_host_hierarchy(tmp_path, monkeypatch, name):
    monkeypatch.setenv("MDP_DEVICE_PRODUCT_TERMS", "1")
    A, b, part = CASES[name]()
    say(f"[products] {name}: n={A.shape[0]} nnz={A.nnz}")
    _same_hierarchy(tmp_path, A, part)


def test_dimension_aware_setup_with_device_products(tmp_path, monkeypatch):
    monkeypatch.setenv("MDP_DEVICE_PRODUCT_TERMS", "1")
    sc = synth.regular_3d(n=16, k_par=1e4, kappa=1e-4, seed=4)
    A, b, part = tpfa.assemble(sc)
    labels = part.astype("int32")
    say("[products] labelled 16^3")
    _same_hierarchy(tmp_path, A, part, labels=labels)


def test_cube100_default_threshold_hierarchy_and_solve(tmp_path):
    """At 100^3 the large products (A P_t, R A, (R A) P on the first levels,
    about 10^7 to 10^8 terms each) run on the device by default: same file,
    same solution bit for bit."""
    os.environ.pop("MDP_DEVICE_PRODUCT_TERMS", None)
    sc = synth.regular_3d(n=100, k_par=1e-4, kappa=1e-4, seed=0)
    A, b, part = tpfa.assemble(sc)
    say("[products] cube 100 default threshold")
    _same_hierarchy(tmp_path, A, part)
    xs = []
    for flags in (0, L.MDP_HOST_PRODUCTS):
        h = L.mdp_setup(A, part, L.mdp_options_default(flags=flags))
        try:
            bt = dev(b)
            x = torch.zeros_like(bt)
            rc, st = L.mdp_solve(h, bt, x)
            assert rc == L.MDP_OK
            xs.append(x)
        finally:
            L.mdp_destroy(h)
    assert torch.equal(xs[0], xs[1])
