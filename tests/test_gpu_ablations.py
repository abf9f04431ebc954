"""The ablation switches' kernel paths against the oracle, through the C ABI.

Every environment switch that selects another kernel or launch shape for the
same operation is read at every launch; each setting here must still give
the oracle's right-hand side (FP64 <= 1e-12, mixed <= 1e-5 per grid
function, max-normalised) and, where the arithmetic is the default's, the
default's values bitwise.  Cases: the BSSN right-hand side with the
cached-load, LDS and async fused kernels, six staging buffers, the plane
order instead of the XCD column walk, and the forced tile shapes; the
constraints with six staging buffers; the wave RK4 step with another
workgroup target.  The grid is ragged (partial tiles in x and y, an odd
number of planes) and wide enough for the column walk."""
import numpy as np
import pytest
import torch

import oracle
from paper_1410_1764_amd import chemora as C
from paper_1410_1764_amd import inputs as I
from tests.helpers import pair, parity
from tests.test_oracle_bssn import _smooth_random

pytestmark = pytest.mark.gpu

N = (45, 27, 11)
TOL = {C.FP64: 1e-12, C.MIXED: 1e-5}
SWITCHES = ("CHEMORA_BSSN_KERNEL", "CHEMORA_BSSN_NBUF", "CHEMORA_BSSN_ORDER",
            "CHEMORA_BSSN_TILE", "CHEMORA_BSSN_SPLIT", "CHEMORA_CONS_NBUF", "CHEMORA_WAVE_WGS")

_cache = {}


def _oracle_rhs():
    if "rhs" not in _cache:
        h = tuple(1.0 / v for v in N)
        _, b = pair(N, 3, h, C.BSSN, slicing=0, shift=1)
        y0 = _smooth_random(N, 51)
        yo = b.embed(y0)
        oracle.fill_periodic(b, yo)
        _cache["rhs"] = (y0, b.interior(oracle.bssn_rhs(b, yo)))
    return _cache["rhs"]


def _clear(monkeypatch):
    for s in SWITCHES:
        monkeypatch.delenv(s, raising=False)


def _gpu_rhs(precision, y0):
    h = tuple(1.0 / v for v in N)
    gr, _ = pair(N, 3, h, C.BSSN, precision=precision, slicing=0, shift=1)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    r = gr.rhs(st)
    torch.cuda.synchronize()
    return gr.download(r)


CASES = [
    # (environment, whether the values must equal the fused single-plane
    # kernel's bitwise (the same point code and staging in other buffers or
    # tiles), or the default's (None: only the workgroup order differs);
    # False: the oracle only (other sources of the staged values))
    ({"CHEMORA_BSSN_KERNEL": "global"}, False),
    ({"CHEMORA_BSSN_KERNEL": "lds"}, False),
    ({"CHEMORA_BSSN_KERNEL": "async", "CHEMORA_BSSN_SPLIT": "0"}, True),
    ({"CHEMORA_BSSN_SPLIT": "0", "CHEMORA_BSSN_NBUF": "6"}, True),
    ({"CHEMORA_BSSN_ORDER": "plane"}, None),
    ({"CHEMORA_BSSN_TILE": "64x4"}, True),
    ({"CHEMORA_BSSN_TILE": "16x16"}, True),
    ({"CHEMORA_BSSN_TILE": "16x8"}, True),
    ({"CHEMORA_BSSN_TILE": "16x4"}, True),
    ({"CHEMORA_BSSN_TILE": "8x8"}, True),
]


@pytest.mark.parametrize("env,fused_arith", CASES,
                         ids=["-".join(f"{k[8:]}={v}" for k, v in e.items()) for e, _ in CASES])
@pytest.mark.parametrize("precision", [C.FP64, C.MIXED])
def test_bssn_rhs_switches(env, fused_arith, precision, monkeypatch):
    y0, ro = _oracle_rhs()
    _clear(monkeypatch)
    default = _gpu_rhs(precision, y0)
    monkeypatch.setenv("CHEMORA_BSSN_SPLIT", "0")
    fused = _gpu_rhs(precision, y0)
    _clear(monkeypatch)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    got = _gpu_rhs(precision, y0)
    e = parity(got, ro)
    print("switch", env, precision, "vs oracle", e.max(), I.BSSN_NAMES[int(np.argmax(e))],
          flush=True)
    assert e.max() <= TOL[precision]
    if fused_arith:
        # the fused point code in another kernel or tile: the fused kernel's values
        assert np.array_equal(got, fused)
    elif fused_arith is None:
        # only the workgroup order differs: the default's values
        assert np.array_equal(got, default)


def test_constraints_six_buffers(monkeypatch):
    h = tuple(1.0 / v for v in N)
    gr, b = pair(N, 3, h, C.BSSN)
    y0 = _smooth_random(N, 53)
    st = gr.upload(y0)
    gr.fill_ghosts(st)
    _clear(monkeypatch)
    hm = gr.new_state()[: 4 * gr.strides[3]].clone()
    norms = gr.constraints(st, hm=hm)
    torch.cuda.synchronize()
    ref_hm, ref_norms = gr.download(hm, nvars=4), norms.cpu().numpy()
    monkeypatch.setenv("CHEMORA_CONS_NBUF", "6")
    hm6 = gr.new_state()[: 4 * gr.strides[3]].clone()
    norms6 = gr.constraints(st, hm=hm6)
    torch.cuda.synchronize()
    yo = b.embed(y0)
    oracle.fill_periodic(b, yo)
    hmo, no = oracle.constraints(b, yo)
    e = parity(gr.download(hm6, nvars=4), b.interior(hmo))
    print("constraints six buffers", e.max(), flush=True)
    assert e.max() <= TOL[C.FP64]
    assert np.array_equal(gr.download(hm6, nvars=4), ref_hm)
    assert np.array_equal(norms6.cpu().numpy(), ref_norms)


@pytest.mark.parametrize("wgs", ["256", "1024", "65536"])
def test_wave_workgroup_target(wgs, monkeypatch):
    n = (70, 37, 23)
    h = tuple(1.0 / v for v in n)
    rng = np.random.default_rng(57)
    y0 = rng.standard_normal((2, n[2], n[1], n[0]))
    gr, b = pair(n, 2, h, C.WAVE)
    dt = 0.25 * min(h)
    _clear(monkeypatch)
    st = gr.upload(y0)
    gr.rk4_step(st, gr.new_workspace(), 0.0, dt, 2)
    torch.cuda.synchronize()
    ref = gr.download(st, ghosts=True)
    monkeypatch.setenv("CHEMORA_WAVE_WGS", wgs)
    st = gr.upload(y0)
    gr.rk4_step(st, gr.new_workspace(), 0.0, dt, 2)
    torch.cuda.synchronize()
    got = gr.download(st, ghosts=True)
    yo = b.embed(y0)
    oracle.rk4(b, oracle.WAVE, oracle.BC_PERIODIC, yo, 0.0, dt, 2)
    e = parity(gr.download(st), b.interior(yo))
    print("wave workgroups", wgs, e.max(), flush=True)
    assert e.max() <= TOL[C.FP64]
    assert np.array_equal(got, ref)
