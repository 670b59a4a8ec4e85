"""GPU parity at the full sizes of the benchmark workloads, on sampled outputs
the oracle computes one by one, and on properties that hold at any size.

* Pusher workload (2^27 particles, 1000 steps, crossed E = -v x B fields and
  uniform-B gyration, gamma log-uniform in [1e2, 1e6]): a random sample is
  pushed by the oracle from the same initial state; the FP64 path matches it
  to rounding, the split-precision path keeps the crossed-field cancellation
  and gamma within FP32 rounding bounds.
* 3D 256x128x128 (8 e-/cell) and 512x256x256 (16 e-/cell, the benchmark's
  own launch configuration): after some steps, the fields E^n, B^n are read
  back into an oracle state and sampled particles are gathered, pushed and
  moved by the oracle; one GPU step must give the same momenta and
  positions (per-particle momentum relative error <= 1e-5 for FP32, 1e-10
  for FP64).
* 256x128x128: discrete continuity residual <= 1e-6 relative on every step
  and the Gauss-law drift at rounding level; the split-precision run agrees
  with the FP64 run in field energy and wake amplitude within 1e-3 over the
  full 2000-step run.
"""
import numpy as np
import pytest

import oracle
from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ pusher
def _push_full(prec, u, Ex, B, cell, off, nsteps, dt):
    dtype = torch.float64 if prec == pic.PIC_FP64 else torch.float32
    n = u.shape[0]
    dev = "cuda"
    tu = torch.from_numpy(np.ascontiguousarray(u.T)).to(dev, dtype).reshape(-1)
    tE = torch.from_numpy(Ex).to(dev, dtype)
    tc = torch.from_numpy(np.ascontiguousarray(cell.T)).to(dev).reshape(-1)
    to = torch.from_numpy(np.ascontiguousarray(off.T)).to(dev, dtype).reshape(-1)
    s = torch.cuda.current_stream()
    pic.pic_push_bench(prec, pic.PIC_VAY, n, nsteps, dt, B, tE.data_ptr(), tu.data_ptr(),
                       tc.data_ptr(), to.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    return tu.view(3, n), tc.view(3, n), to.view(3, n), tE


def _sample_rows(t3n, idx):
    return t3n[:, torch.from_numpy(idx).to(t3n.device)].double().cpu().numpy().T


@pytest.mark.parametrize("kind", ["crossed", "gyration"])
def test_pusher_full_size_sampled(kind):
    n, nsteps, dt = 1 << 27, 1000, workloads.PUSH_DT
    u, Ex, B, cell, off = workloads.pusher_set(n, kind, seed=2 if kind == "crossed" else 3)
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(n, size=4096, replace=False))
    # oracle on the sample, from the state each precision starts from
    E = np.zeros((idx.size, 3))
    E[:, 0] = Ex[idx]
    Bn = np.tile(B, (idx.size, 1))
    for prec in (pic.PIC_FP64, pic.PIC_FP32_SPLIT):
        if prec == pic.PIC_FP32_SPLIT:
            u0 = u[idx].astype(np.float32).astype(np.float64)
            E0 = E.astype(np.float32).astype(np.float64)
            pos0 = cell[idx] + off[idx].astype(np.float32).astype(np.float64)
        else:
            u0, E0, pos0 = u[idx], E, cell[idx] + off[idx]
        uo, po = oracle.push_many(u0, E0, Bn, pos0, dt, nsteps)
        tu, tc, to, tE = _push_full(prec, u, Ex, B, cell, off, nsteps, dt)
        ug = _sample_rows(tu, idx)
        pg = _sample_rows(tc, idx) + _sample_rows(to, idx)
        del tu, tc, to, tE
        _free()
        rel = np.linalg.norm(ug - uo, axis=1) / np.linalg.norm(uo, axis=1)
        print(f"\n{kind} prec={prec}: max |u - u_oracle|/|u| = {rel.max():.3e}")
        if prec == pic.PIC_FP64:
            assert rel.max() < 1e-10
            assert np.abs(pg - po).max() < 1e-6
        elif kind == "crossed":
            # E + v x B = 0: the momentum stays what it was (FP32 storage of a
            # constant vector, up to a random walk of rounding)
            cancel = np.linalg.norm(ug - u0, axis=1) / np.linalg.norm(u0, axis=1)
            print(f"crossed FP32 cancellation {cancel.max():.3e}")
            # a random walk of half an FP32 ulp per step: sqrt(N) 2^-24 ~ 1.9e-6
            assert cancel.max() < 1e-5
            assert rel.max() < 1e-5
        else:
            g0 = np.sqrt(1 + (u0**2).sum(1))
            g1 = np.sqrt(1 + (ug**2).sum(1))
            drift = (np.abs(g1 - g0) / g0).max()
            print(f"gyration FP32 gamma drift {drift:.3e}")
            assert drift < 1.5 * nsteps * 2.0**-23
            # the phase error grows by at most ~2^-24 per step
            assert rel.max() < 4.0 * nsteps * 2.0**-24


# ------------------------------------------------------------------ PIC step
def _oracle_fields(cfg, run):
    """An oracle state on the run's grid holding the run's E^n and B^n."""
    st = oracle.State(dict(cfg, ppc=0))
    for c in range(6):
        st.field(c)[...] = run.field(c)
    return st


def _read_blocks(run, firsts, count):
    parts = [run.particles(f, count) for f in firsts]
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def _sampled_step(cfg, prec, steps_before, nblocks=16, block=1024, seed=7):
    """One GPU step against the oracle's gather, push and move of a sample."""
    run = pic.Run(cfg, prec)
    every = cfg.get("sort_every", 20)
    assert (steps_before % every) != 0, "the sampled step must not sort (slots stay put)"
    run.step(steps_before)
    slots, _ = pic.pic_particle_count(run.handle)
    rng = np.random.default_rng(seed)
    firsts = np.sort(rng.choice(max(1, slots // block), size=nblocks, replace=False)) * block
    p0 = _read_blocks(run, firsts, block)
    st = _oracle_fields(cfg, run)
    run.step(1)
    p1 = _read_blocks(run, firsts, block)
    d = run.derived
    dt = d["dt"]
    run.close()
    _free()
    o0 = np.argsort(p0["id"])
    o1 = np.argsort(p1["id"])
    ids, i0, i1 = np.intersect1d(p0["id"][o0], p1["id"][o1], assume_unique=True, return_indices=True)
    a = {k: v[o0][i0] for k, v in p0.items()}
    b = {k: v[o1][i1] for k, v in p1.items()}
    assert ids.size > 0.98 * p0["id"].size
    Lx, Ly = cfg["nx"] * cfg["dx"], cfg["ny"] * cfg["dy"]
    urel, perr = [], []
    for q in range(ids.size):
        E, B = st.gather(a["z"][q], a["x"][q], a["y"][q])
        u = oracle.push([a["ux"][q], a["uy"][q], a["uz"][q]], E, B, -0.5 * dt)
        g = np.sqrt(1.0 + u @ u)
        z1 = a["z"][q] + dt * u[2] / g
        x1 = a["x"][q] + dt * u[0] / g
        y1 = a["y"][q] + dt * u[1] / g
        ug = np.array([b["ux"][q], b["uy"][q], b["uz"][q]])
        urel.append(np.linalg.norm(ug - u) / np.linalg.norm(u))
        dx_ = (b["x"][q] - x1 + 0.5 * Lx) % Lx - 0.5 * Lx
        dy_ = (b["y"][q] - y1 + 0.5 * Ly) % Ly - 0.5 * Ly
        perr.append(max(abs(b["z"][q] - z1), abs(dx_), abs(dy_)))
    st.close()
    return np.array(urel), np.array(perr), ids.size


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_step_sampled_256x128x128(prec):
    cfg = workloads.config("c3")
    urel, perr, n = _sampled_step(cfg, prec, steps_before=7)
    print(f"\n256x128x128 {prec}: {n} particles, max du/u {urel.max():.3e}, max dx {perr.max():.3e}")
    if prec == "fp32":
        assert urel.max() <= 1e-5
        assert perr.max() <= 1e-5 * cfg["dz"]
    else:
        assert urel.max() <= 1e-10
        assert perr.max() <= 1e-10 * cfg["dz"]


def test_step_sampled_512x256x256_bench_configuration():
    cfg = workloads.config("c5")
    urel, perr, n = _sampled_step(cfg, "fp32", steps_before=12)
    print(f"\n512x256x256 fp32: {n} particles, max du/u {urel.max():.3e}, max dx {perr.max():.3e}")
    assert urel.max() <= 1e-5
    assert perr.max() <= 1e-5 * cfg["dz"]


def test_continuity_and_gauss_256x128x128_fp32():
    cfg = workloads.config("c3")
    run = pic.Run(cfg, "fp32", continuity=True)
    worst = 0.0
    for _ in range(6):
        run.step(1)
        d = run.diag(pic.PIC_DIAG_FIELDS)
        worst = max(worst, d["cont_resid"])
    d = run.diag()
    run.close()
    _free()
    print(f"\n256x128x128 fp32: continuity {worst:.3e}, gauss drift {d['gauss_drift']:.3e}")
    assert worst <= 1e-6
    assert d["gauss_drift"] <= 1e-5


def test_fp32_vs_fp64_energy_and_wake_256x128x128_full_run():
    cfg = workloads.config("c3")
    out = {}
    for prec in ("fp64", "fp32"):
        run = pic.Run(cfg, prec)
        for _ in range(cfg["steps"] // 500):
            run.step(500)
            run.synchronize()
            print(f"\n{prec} step {run.diag(0)['step']}", flush=True)
        out[prec] = run.diag()
        run.close()
        _free()
    a, b = out["fp32"], out["fp64"]
    print({k: (a[k], b[k]) for k in ("U_E", "U_B", "Ez_max", "KE", "n_particles")})
    assert a["step"] == b["step"] == cfg["steps"]
    for k in ("U_E", "U_B", "Ez_max"):
        assert a[k] == pytest.approx(b[k], rel=1e-3), k
