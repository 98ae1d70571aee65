"""Parity at the full workload sizes (256^3 and 512^3 complex128, 512^3 and
1024^3 complex64), in the launch configuration the benchmark times (default
plan, out of place).

256^3 and 512^3 complex128 are compared against the full recursive oracle;
every size is also checked on sampled output lines computed one by one from
the definition (X[ka, kb, :] for chosen ka, kb), and by Parseval and the
normalised round trip, which hold at any size.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1501_07350_amd as offt
import synth

pytestmark = pytest.mark.gpu

C128, C64 = torch.complex128, torch.complex64
LINES = [(0, 0), (1, 0), (0, 1), (5, 7), (17, 3), (-1, -1), (-2, 11), (100, -3)]


def check_size(n, dtype, full_oracle):
    shape = (n, n, n)
    print(f"case {shape} {dtype}", flush=True)
    x = synth.complex_grid(shape, dtype, device="cuda")
    plan = offt.Plan(shape, dtype=dtype, normalize_inverse=True)
    y = plan.forward(x)
    torch.cuda.synchronize()
    tol = oracle.tolerance(x.numel(), dtype == C64)
    xh = x.cpu().numpy().astype(np.complex128)
    yh = y.cpu().numpy().astype(np.complex128)
    # sampled lines from the definition
    got, ref = [], []
    for ka, kb in LINES:
        ka %= n
        kb %= n
        ref.append(oracle.dft3_line(xh, ka, kb))
        got.append(yh[ka, kb])
    e_lines = oracle.rel_l2(np.concatenate(got), np.concatenate(ref))
    # Parseval: ||X||^2 = N ||x||^2
    e_pars = abs(np.sum(np.abs(yh) ** 2) / (xh.size * np.sum(np.abs(xh) ** 2)) - 1.0)
    e_full = oracle.rel_l2(yh, oracle.fft3(xh)) if full_oracle else float("nan")
    del yh
    z = plan.backward(y)
    torch.cuda.synchronize()
    e_rt = oracle.rel_l2(z.cpu().numpy(), xh)
    print(f"{shape} {dtype}: lines {e_lines:.2e} parseval {e_pars:.2e} full {e_full:.2e} "
          f"roundtrip {e_rt:.2e} tol {tol:.1e} plan {plan.describe()}", flush=True)
    assert e_lines <= tol and e_rt <= tol and e_pars <= tol
    if full_oracle:
        assert e_full <= tol


def test_256_complex128_full_oracle():
    check_size(256, C128, True)


def test_512_complex128_full_oracle():
    check_size(512, C128, True)


def test_512_complex64_sampled():
    check_size(512, C64, False)


def test_1024_complex64_sampled():
    check_size(1024, C64, False)
