"""Helpers of the GPU parity tests: build states on the device, read them
back, run the FP64 oracle on the same bytes, and compare to the stated
tolerances."""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np
import torch

import oracle
import synth

DEV = torch.device("cuda:0")

# FP32 path: attributes within 1e-6 of the oracle (unit-floor relative error).
TOL_THETA = 1e-6
# FP32 moments: relative error with the group's RMS as floor.
TOL_MOMENT = 1e-6
# BF16 moments: within one bf16 unit in the last place of the FP64 value
# (2^-7 relative at most), plus the FP32 arithmetic's own share.
TOL_BF16 = 2.0 ** -7 * 1.001


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@dataclass
class GpuState:
    groups: list                 # paper_2601_16736_amd.Group
    spec: list                   # (name, dim, lr, dar_kind)
    t: torch.Tensor
    bf16: bool

    def host(self) -> Dict[str, Dict[str, np.ndarray]]:
        out = {}
        for (name, *_), g in zip(self.spec, self.groups):
            d = {"param": g.param.cpu().numpy().copy(), "grad": g.grad.cpu().numpy().copy()}
            for k, tens in (("m", g.exp_avg), ("v", g.exp_avg_sq)):
                if self.bf16:
                    d[k] = bf16_bits_to_f64(tens.view(torch.int16).cpu().numpy().view(np.uint16))
                else:
                    d[k] = tens.cpu().numpy().astype(np.float64)
            out[name] = d
        out["_t"] = self.t.cpu().numpy().copy()
        return out


def make_state(gs, n: int, spec, seed: int, bf16: bool = False, dar_lambda=None, dar_clip: float = 10.0,
               reg_mode: int = 0, nonzero_state: bool = True) -> GpuState:
    """Random attributes and (optionally) moments/step counts already in use."""
    r = synth.rng(seed, 100)
    groups = []
    for name, dim, lr, dar in spec:
        p = torch.from_numpy(r.standard_normal((n, dim), dtype=np.float32)).to(DEV)
        g = torch.zeros((n, dim), dtype=torch.float32, device=DEV)
        if nonzero_state:
            m = torch.from_numpy((1e-4 * r.standard_normal((n, dim))).astype(np.float32))
            v = torch.from_numpy((1e-6 * r.random((n, dim)) + 1e-9).astype(np.float32))
        else:
            m = torch.zeros((n, dim), dtype=torch.float32)
            v = torch.zeros((n, dim), dtype=torch.float32)
        mdt = torch.bfloat16 if bf16 else torch.float32
        lam = (1e-3 if dar == 1 else 1e-5) if dar_lambda is None else dar_lambda
        groups.append(gs.Group(p, g, m.to(mdt).to(DEV), v.to(mdt).to(DEV), lr, dar_kind=dar,
                               dar_lambda=lam if dar else 0.0, dar_clip=dar_clip, reg_mode=reg_mode))
    t = torch.from_numpy(r.integers(0, 50, n).astype(np.int32) if nonzero_state else np.zeros(n, np.int32)).to(DEV)
    return GpuState(groups, list(spec), t, bf16)


def set_grads(state: GpuState, mask: np.ndarray, seed: int, step: int, poison_invisible: bool = True) -> None:
    n = state.t.shape[0]
    gr = synth.grads(n, state.spec, mask, seed, step)
    for (name, *_), g in zip(state.spec, state.groups):
        a = gr[name]
        if poison_invisible:
            a = a.copy()
            a[mask == 0] = np.nan
        g.grad.copy_(torch.from_numpy(a))


def oracle_groups(host, spec, groups) -> List[oracle.Group]:
    out = []
    for (name, dim, lr, dar), g in zip(spec, groups):
        h = host[name]
        out.append(oracle.Group(h["param"].astype(np.float64), h["grad"].astype(np.float64),
                                h["m"].astype(np.float64).copy(), h["v"].astype(np.float64).copy(), lr,
                                dar_kind=dar, dar_lambda=g.dar_lambda, dar_clip=g.dar_clip,
                                reg_mode=g.reg_mode))
    return out


def oracle_config(cfg, reg_norm: float = 1e5) -> oracle.Config:
    return oracle.Config(beta1=cfg.beta1, beta2=cfg.beta2, eps=cfg.eps, reg_norm=cfg.reg_norm, seed=cfg.seed,
                         iteration=cfg.iteration, rsr_enable=cfg.rsr_enable, rsr_alpha1=cfg.rsr_alpha1,
                         rsr_alpha2=cfg.rsr_alpha2, rsr_ratio=cfg.rsr_ratio)


def theta_err(x: np.ndarray, r: np.ndarray) -> float:
    if x.size == 0:
        return 0.0
    return float(np.max(np.abs(x.astype(np.float64) - r) / np.maximum(np.abs(r), 1.0)))


def moment_err(x: np.ndarray, r: np.ndarray, rows: np.ndarray) -> float:
    """Relative error with the RMS of the changed rows as floor."""
    if x.size == 0:
        return 0.0
    ref = r[rows] if rows is not None and rows.any() else r
    rms = float(np.sqrt(np.mean(ref * ref))) if ref.size else 0.0
    floor = max(rms, 1e-30)
    return float(np.max(np.abs(x.astype(np.float64) - r) / np.maximum(np.abs(r), floor)))


def compare(after: dict, before: dict, ogroups, spec, t_ref: np.ndarray, touched: np.ndarray, bf16: bool,
            label: str = "") -> Dict[str, float]:
    """after/before: GpuState.host() dicts; ogroups: oracle groups after the
    step; touched: rows the step may change (visible or RSR-sampled)."""
    np.testing.assert_array_equal(after["_t"], t_ref, err_msg=f"{label} step counts")
    errs = {}
    for (name, dim, *_), O in zip(spec, ogroups):
        A, B = after[name], before[name]
        untouched = ~touched
        np.testing.assert_array_equal(A["param"][untouched], B["param"][untouched],
                                      err_msg=f"{label} {name}: untouched theta changed")
        np.testing.assert_array_equal(A["m"][untouched], B["m"][untouched], err_msg=f"{label} {name}: m changed")
        np.testing.assert_array_equal(A["v"][untouched], B["v"][untouched], err_msg=f"{label} {name}: v changed")
        e_t = theta_err(A["param"], O.param)
        assert e_t <= TOL_THETA, f"{label} {name}: theta max rel err {e_t:.3e} > {TOL_THETA}"
        if bf16:
            for k, ref in (("m", O.m), ("v", O.v)):
                d = np.abs(A[k] - ref)
                # one bf16 ulp of the value, plus the FP32 arithmetic's error,
                # which scales with the terms (the RMS) when m cancels
                sub = ref[touched] if touched.any() else ref
                rms = float(np.sqrt(np.mean(sub * sub))) if sub.size else 0.0
                bound = TOL_BF16 * np.abs(ref) + TOL_MOMENT * rms + 1e-38
                bad = d > bound
                assert not bad.any(), (f"{label} {name}.{k}: {bad.sum()} elements beyond one bf16 ulp, e.g. "
                                       f"{A[k][bad][:3]} vs {ref[bad][:3]}")
            e_m = float(np.max(np.abs(A["m"] - O.m) / np.maximum(np.abs(O.m), 1e-30)))
            e_v = float(np.max(np.abs(A["v"] - O.v) / np.maximum(np.abs(O.v), 1e-30)))
        else:
            e_m = moment_err(A["m"], O.m, touched)
            e_v = moment_err(A["v"], O.v, touched)
            assert e_m <= TOL_MOMENT, f"{label} {name}: m err {e_m:.3e}"
            assert e_v <= TOL_MOMENT, f"{label} {name}: v err {e_v:.3e}"
        errs[name] = max(e_t, 0.0)
    return errs


def rsr_sampled_mask(n: int, seed: int, iteration: int, ratio: float) -> np.ndarray:
    return oracle.rsr_sample_mask(seed, iteration, n, ratio)
