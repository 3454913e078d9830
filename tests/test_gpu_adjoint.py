"""GPU parity of the hand-written adjoint (step, observables, init, trajectory)
against the FP64 oracle's reverse mode and against central finite differences
of the GPU forward, through the C ABI."""

import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import gradient as G
from oracle import lbm as OL
import workloads as W
import paper_2107_14774_amd as P
from paper_2107_14774_amd import adjoint as ADJ
from helpers import fp32_rounded_state, gpu_lattice, oracle_params, random_state, rel_l2

pytestmark = pytest.mark.gpu
DT = torch.float64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


ADJ_CASES = [
    ("periodic_ragged_local", (300, 5, 4), 1.0, 0.5, "periodic", "periodic", "local"),
    ("duct_walls_local", (19, 10, 8), 1.0, 0.25, "bounceback", "bounceback", "local"),
    ("aniso_lowmach", (16, 9, 12), 0.5, 0.25, "periodic", "bounceback", "lowmach"),
    ("walls_off", (12, 7, 6), 0.8, 1.2, "bounceback", "periodic", "off"),
    ("x_walls_local", (11, 6, 5), 0.5, 1.0, "bounceback", "bounceback", "local", "bounceback"),
    ("cavity_moving_faces", (9, 8, 7), 0.5, 1.0, "bounceback", "bounceback", "local", "bounceback",
     ((0, 0, 0), (0, 0, 0), (0, 0, 0), (0.05, 0, 0.02), (0.03, 0.01, 0), (0, 0, 0))),
    ("raw_periodic_local", (70, 5, 4), 1.0, 0.5, "periodic", "periodic", "local", "periodic",
     ((0, 0, 0),) * 6, "raw"),
    ("raw_duct_lowmach", (13, 9, 8), 0.5, 0.25, "bounceback", "bounceback", "lowmach", "periodic",
     ((0, 0, 0),) * 6, "raw"),
]


@pytest.mark.parametrize("case", ADJ_CASES, ids=[c[0] for c in ADJ_CASES])
def test_step_adjoint_matches_oracle_vjp(case):
    name, (nx, ny, nz), r, s, by, bz, corr = case[:7]
    bx = case[7] if len(case) > 7 else "periodic"
    wv = case[8] if len(case) > 8 else ((0, 0, 0),) * 6
    moments = case[9] if len(case) > 9 else "central"
    _say("case", name)
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.27, corr=corr, bc_y=by, bc_z=bz, bc_x=bx,
                      wall_velocity=wv, moments=moments)
    f0 = fp32_rounded_state(random_state(p, 21), p)
    g = np.random.Generator(np.random.PCG64(22))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32)
    lam_f = torch.tensor(g.standard_normal((27, *p.shape)))
    lat = gpu_lattice(p)
    st = lat.new_state()
    lat.import_populations(st, f0.cuda())
    lam_in = lat.new_adjoint()
    lam_out = lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, lam_f.cuda(), lam_in)
    gF = torch.zeros((3, *p.shape), dtype=torch.float32, device="cuda")
    gFu = torch.zeros(3, dtype=torch.float64, device="cuda")
    P.lbm_step_adjoint(lat.h, st, lam_in, lam_out, force.cuda(), gF, gFu)
    got = torch.empty((27, *p.shape), dtype=DT, device="cuda")
    P.lbm_adjoint_to_natural(lat.h, lam_out, got)
    want_f, want_F = G.step_vjp(f0, p, force.to(DT), lam_f)
    err = (got.cpu() - want_f).abs().max().item() / want_f.abs().max().item()
    errF = (gF.cpu().to(DT) - want_F).abs().max().item() / want_F.abs().max().item()
    errU = (gFu.cpu() - want_F.reshape(3, -1).sum(-1)).abs().max().item() / want_F.reshape(3, -1).sum(-1).abs().max().item()
    _say(f"{name}: rel max err lambda {err:.2e}, force grad {errF:.2e}, uniform force grad {errU:.2e}")
    assert err < 2e-6
    assert errF < 2e-5
    assert errU < 1e-4


def test_adjoint_natural_roundtrip():
    p = oracle.Params(9, 6, 5, r=1.0, s=0.5, bc_y="bounceback")
    lat = gpu_lattice(p)
    nat = torch.randn((27, *p.shape), dtype=DT, device="cuda")
    slots = lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, nat, slots)
    back = torch.empty_like(nat)
    P.lbm_adjoint_to_natural(lat.h, slots, back)
    assert torch.equal(back, nat.to(torch.float32).to(DT))


def test_moments_and_init_adjoint_match_oracle():
    p = oracle.Params(13, 7, 6, r=0.8, s=0.5, bc_z="bounceback")
    f0 = fp32_rounded_state(random_state(p, 31), p)
    g = np.random.Generator(np.random.PCG64(32))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32)
    g_rho = torch.tensor(g.standard_normal(p.shape)).to(torch.float32)
    g_u = torch.tensor(g.standard_normal((3, *p.shape))).to(torch.float32)
    lat = gpu_lattice(p)
    st = lat.new_state()
    lat.import_populations(st, f0.cuda())
    adj = lat.new_adjoint()
    gF = torch.zeros((3, *p.shape), dtype=torch.float32, device="cuda")
    P.lbm_moments_adjoint(lat.h, st, adj, force.cuda(), g_rho.cuda(), g_u.cuda(), gF)
    got = torch.empty((27, *p.shape), dtype=DT, device="cuda")
    P.lbm_adjoint_to_natural(lat.h, adj, got)
    want = G.observables_vjp(f0, p, force.to(DT), g_rho.to(DT), g_u.to(DT))
    err = (got.cpu() - want).abs().max().item() / want.abs().max().item()
    _say(f"moments adjoint rel err {err:.2e}")
    assert err < 1e-6
    # force part of the observables: d u / d F = 1 / (2 rho)
    rho, _ = OL.observables(f0, p, force.to(DT))
    assert torch.allclose(gF.cpu().to(DT), 0.5 * g_u.to(DT) / rho, rtol=1e-5, atol=1e-9)
    # init adjoint
    rho0 = torch.tensor(1.0 + 0.01 * g.standard_normal(p.shape))
    u0 = torch.tensor(0.02 * g.standard_normal((3, *p.shape)))
    lam = torch.tensor(g.standard_normal((27, *p.shape))).to(torch.float32)
    slots = lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, lam.to(DT).cuda(), slots)
    gr = torch.empty(p.shape, dtype=DT, device="cuda")
    gu = torch.empty((3, *p.shape), dtype=DT, device="cuda")
    P.lbm_init_adjoint(lat.h, slots, rho0.cuda(), u0.cuda(), gr, gu)
    wr, wu = G.init_vjp(rho0, u0, p, lam.to(DT))
    e1 = (gr.cpu() - wr).abs().max().item() / wr.abs().max().item()
    e2 = (gu.cpu() - wu).abs().max().item() / wu.abs().max().item()
    _say(f"init adjoint rel err rho {e1:.2e}, u {e2:.2e}")
    assert e1 < 1e-12 and e2 < 1e-12


def _loss_gpu(lat, u0, force, target, nsteps, every):
    u = ADJ.simulate(lat, u0, force, nsteps, every)
    return 0.5 * ((u.to(DT) - target) ** 2).sum(), u


def test_trajectory_gradient_matches_oracle_on_replica():
    """dL/dF and dL/du0 through 24 steps on a 12x10x8 replica of the adjoint duct workload."""
    w = W.ADJOINT_DUCT_128
    p = oracle_params(w, nx=12, ny=10, nz=8)
    g = np.random.Generator(np.random.PCG64(41))
    force = torch.tensor(1e-5 * g.standard_normal((3, *p.shape))).to(torch.float32)
    u0 = torch.tensor(1e-3 * g.standard_normal((3, *p.shape)))
    target = torch.tensor(1e-3 * g.standard_normal((3, *p.shape)))
    nsteps = 24
    L_o, gF_o, gu_o = G.loss_and_gradients(p, torch.ones(p.shape, dtype=DT), u0, force.to(DT), target, nsteps)
    lat = gpu_lattice(p)
    uc = u0.cuda().requires_grad_(True)
    Fc = force.cuda().requires_grad_(True)
    L_g, _ = _loss_gpu(lat, uc, Fc, target.cuda(), nsteps, 5)
    L_g.backward()
    eF = rel_l2(Fc.grad.cpu(), gF_o)
    eu = rel_l2(uc.grad.cpu(), gu_o)
    _say(f"replica trajectory: loss rel err {abs(L_g.item() - L_o.item()) / L_o.item():.2e}, "
         f"dL/dF rel L2 {eF:.2e}, dL/du0 rel L2 {eu:.2e}")
    assert eF < 1e-4 and eu < 1e-4


@pytest.mark.parametrize("storage", ["f32", "bf16_sr"])
def test_checkpoint_interval_does_not_change_gradient(storage):
    """Checkpoint intervals and nested recomputation (max_states < K) give bitwise-equal gradients.
    With stochastic rounding (BF16-SR) this also checks that every recomputed segment takes the step
    counters of the forward pass, so it reproduces the forward states bit for bit."""
    w = W.ADJOINT_DUCT_128
    p = oracle_params(w, nx=24, ny=12, nz=10)
    g = np.random.Generator(np.random.PCG64(42))
    force = torch.tensor(1e-5 * g.standard_normal((3, *p.shape))).to(torch.float32).cuda()
    target = torch.tensor(1e-3 * g.standard_normal((3, *p.shape))).cuda()
    u0 = torch.zeros((3, *p.shape), dtype=DT, device="cuda")
    lat = gpu_lattice(p, storage=storage)
    grads = []
    for every, cap in ((1, 128), (7, 128), (40, 128), (40, 3), (25, 4)):
        Fc = force.clone().requires_grad_(True)
        P.lbm_set_step_counter(lat.h, 1000)
        u = ADJ.simulate(lat, u0, Fc, 40, every, max_states=cap)
        assert lat.h.step_counter == 1040                  # the backward leaves the counter where the forward did
        (0.5 * ((u.to(DT) - target) ** 2).sum()).backward()
        grads.append(Fc.grad.clone())
    for gr in grads[1:]:
        assert torch.equal(grads[0], gr)


def test_full_size_duct_gradient_vs_central_differences():
    """Adjoint workload at full size: 128x128x64 duct, 500 steps, checkpoint every 50;
    dL/dF on 16 seeded entries vs central differences of the GPU forward."""
    w = W.ADJOINT_DUCT_128
    p = oracle_params(w)
    force = torch.from_numpy(W.body_force_field(w)).to(torch.float32).cuda()
    target = torch.from_numpy(W.target_velocity(w)).cuda()
    u0 = torch.zeros((3, *p.shape), dtype=DT, device="cuda")
    lat = gpu_lattice(p)
    Fc = force.clone().requires_grad_(True)
    L_g, _ = _loss_gpu(lat, u0, Fc, target, w.steps, w.extra["checkpoint"])
    L_g.backward()
    grad = Fc.grad
    idx = W.sample_indices(w.extra["fd_entries"], force.numel(), w.extra["fd_seed"])
    h = 1e-5
    worst = 0.0
    scale = grad.abs().max().item()
    with torch.no_grad():
        for flat in idx:
            c = np.unravel_index(int(flat), force.shape)
            Fp, Fm = force.clone(), force.clone()
            Fp[c] += h
            Fm[c] -= h
            lp, _ = _loss_gpu(lat, u0, Fp, target, w.steps, w.steps)
            lm, _ = _loss_gpu(lat, u0, Fm, target, w.steps, w.steps)
            fd = ((lp - lm) / (2 * h)).item()
            ad = grad[c].item()
            worst = max(worst, abs(fd - ad) / scale)
            _say(f"entry {c}: adjoint {ad:.6e} fd {fd:.6e}")
    _say(f"full-size duct: worst |fd - adjoint| / max|grad| = {worst:.2e}")
    assert worst < 1e-3


FULL_ADJ_CASES = [
    # name, grid, r, s, (bc_x, bc_y, bc_z), moving walls, moments, storage, force field, gather kind override
    ("full_periodic_field_f32", (40, 6, 5), 1.0, 0.5, ("periodic",) * 3, None, "central", "f32", True, None),
    ("full_duct_f32", (19, 10, 8), 1.0, 0.25, ("periodic", "bounceback", "bounceback"), None, "central", "f32",
     False, None),
    ("full_box_moving_faces_f32", (9, 8, 7), 0.5, 1.0, ("bounceback",) * 3,
     ((0, 0, 0), (0, 0, 0), (0, 0, 0), (0.05, 0, 0.02), (0.03, 0.01, 0), (0, 0, 0)), "central", "f32", False, None),
    ("full_raw_aniso_f16", (16, 9, 12), 0.5, 0.25, ("periodic", "periodic", "bounceback"), None, "raw", "f16",
     True, None),
    ("full_duct_64bit_slots", (13, 9, 8), 0.75, 1.0, ("bounceback",) * 3, None, "central", "f32", True, "2"),
    # one-node and three-node axes: the stencil and its transpose wrap onto the node itself
    ("full_thin_axes_f32", (3, 1, 17), 1.0, 0.5, ("periodic", "periodic", "bounceback"), None, "central", "f32",
     True, None),
    ("full_duct_bf16", (18, 7, 6), 1.0, 0.5, ("periodic", "bounceback", "bounceback"), None, "central", "bf16",
     True, None),
]


def _full_case(case, corr="full"):
    """Oracle parameters and a GPU lattice for one of FULL_ADJ_CASES."""
    import os
    name, (nx, ny, nz), r, s, (bx, by, bz), wv, moments, storage, field, kind = case
    p = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.27, corr=corr, bc_x=bx, bc_y=by, bc_z=bz,
                      wall_velocity=wv or ((0, 0, 0),) * 6, moments=moments)
    old = os.environ.get("LBM_GATHER_KIND")
    if kind:
        os.environ["LBM_GATHER_KIND"] = kind
    try:
        lat = gpu_lattice(p, storage=storage)
    finally:
        if old is None:
            os.environ.pop("LBM_GATHER_KIND", None)
        else:
            os.environ["LBM_GATHER_KIND"] = old
    return p, lat


@pytest.mark.parametrize("case", FULL_ADJ_CASES, ids=[c[0] for c in FULL_ADJ_CASES])
def test_full_corrections_step_adjoint_matches_oracle_vjp(case):
    """lbm_step_adjoint_full: one reverse step of the full corrections (exact time level) against the
    oracle's reverse mode, which differentiates the density gradient's stencil as well."""
    name, (nx, ny, nz), r, s, (bx, by, bz), wv, moments, storage, field, kind = case
    _say("case", name)
    p, lat = _full_case(case)
    f0 = fp32_rounded_state(random_state(p, 31), p)
    g = np.random.Generator(np.random.PCG64(32))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32) if field else None
    lam_f = torch.tensor(g.standard_normal((27, *p.shape)))
    st = lat.new_state()
    lat.import_populations(st, f0.cuda())
    f_in = lat.export_populations(st).cpu()            # the stored (for FP16: rounded) start
    lam_in, lam_out = lat.new_adjoint(), lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, lam_f.cuda(), lam_in)
    drho, gw = lat.field(1), lat.field(3)
    gF = torch.zeros((3, *p.shape), dtype=torch.float32, device="cuda")
    gFu = torch.zeros(3, dtype=torch.float64, device="cuda")
    fc = force.cuda() if field else None
    P.lbm_step_adjoint_full(lat.h, st, lam_in, lam_out, drho, gw, fc, gF, gFu)
    got = torch.empty((27, *p.shape), dtype=DT, device="cuda")
    P.lbm_adjoint_to_natural(lat.h, lam_out, got)
    force_o = force.to(DT) if field else torch.zeros((3, *p.shape), dtype=DT)
    want_f, want_F = G.step_vjp(f_in, p, force_o, lam_f.to(torch.float32).to(DT))
    err = (got.cpu() - want_f).abs().max().item() / want_f.abs().max().item()
    errF = (gF.cpu().to(DT) - want_F).abs().max().item() / want_F.abs().max().item()
    sumF = want_F.reshape(3, -1).sum(-1)
    errU = (gFu.cpu() - sumF).abs().max().item() / sumF.abs().max().item()
    # the part of the result that comes from the density gradient alone, for scale
    p_loc = oracle.Params(nx, ny, nz, r=r, s=s, omega_nu=1.45, omega_xi=1.27, corr="local", bc_x=bx, bc_y=by,
                          bc_z=bz, wall_velocity=wv or ((0, 0, 0),) * 6, moments=moments)
    want_loc, _ = G.step_vjp(f_in, p_loc, force_o, lam_f.to(torch.float32).to(DT))
    share = (want_f - want_loc).abs().max().item() / want_f.abs().max().item()
    _say(f"{name}: rel max err lambda {err:.2e} (the full terms change it by {share:.2e}), force grad {errF:.2e}, "
         f"uniform force grad {errU:.2e}")
    assert err < 2e-6 and share > 50 * err
    assert errF < 2e-5
    assert errU < 1e-4


@pytest.mark.parametrize("case", [FULL_ADJ_CASES[1], FULL_ADJ_CASES[3]], ids=[FULL_ADJ_CASES[1][0], FULL_ADJ_CASES[3][0]])
def test_full_corrections_exact_drho_mode_equals_exact(case):
    """Mode "exact_drho" (the state's density supplied, as lbm_density writes it) gives the exact level's
    results bit for bit without its density pass."""
    name, (nx, ny, nz), r, s, (bx, by, bz), wv, moments, storage, field, kind = case
    p, lat = _full_case(case)
    f0 = fp32_rounded_state(random_state(p, 35), p)
    g = np.random.Generator(np.random.PCG64(36))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32).cuda() if field else None
    lam_f = torch.tensor(g.standard_normal((27, *p.shape)))
    st = lat.new_state()
    lat.import_populations(st, f0.cuda())
    lam_in = lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, lam_f.cuda(), lam_in)
    outs = []
    for mode in ("exact", "exact_drho"):
        drho = lat.density(st) if mode == "exact_drho" else lat.field(1)
        lam_out, gw = lat.new_adjoint(), lat.field(3)
        gF = torch.zeros((3, *p.shape), dtype=torch.float32, device="cuda")
        gFu = torch.zeros(3, dtype=torch.float64, device="cuda")
        P.lbm_step_adjoint_full(lat.h, st, lam_in, lam_out, drho, gw, force, gF, gFu, mode=mode)
        outs.append((lam_out, gw, gF, gFu))
    for a, b in zip(outs[0][:3], outs[1][:3]):
        assert torch.equal(a, b)
    # the uniform-force gradient sums block totals with atomics, in any order
    assert torch.allclose(outs[0][3], outs[1][3], rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("case", FULL_ADJ_CASES, ids=[c[0] for c in FULL_ADJ_CASES])
def test_full_corrections_lagged_step_adjoint_matches_oracle_vjp(case):
    """lbm_step_adjoint_full at the lagged time level: the gradient comes from the density D of another
    state, so lambda(t) = (d step / d f)^T lambda(t+1) at fixed D, plus the stencil transpose of the pending
    cotangent gp of the next step's gradient (taken from this state's density); grad_work receives the
    cotangent of D's gradient, which lbm_density_adjoint carries back to every population of that state.
    Oracle: reverse mode of <lambda, step(f, grad_from=D)> + <gp, grad(rho(f))>."""
    name, (nx, ny, nz), r, s, (bx, by, bz), wv, moments, storage, field, kind = case
    _say("case", name, "(lagged)")
    p, lat = _full_case(case)
    f0 = fp32_rounded_state(random_state(p, 31), p)
    fD = fp32_rounded_state(random_state(p, 33), p)
    g = np.random.Generator(np.random.PCG64(34))
    force = torch.tensor(1e-4 * g.standard_normal((3, *p.shape))).to(torch.float32) if field else None
    lam_f = torch.tensor(g.standard_normal((27, *p.shape))).to(torch.float32)
    gp = torch.tensor(g.standard_normal((3, *p.shape))).to(torch.float32)
    st, stD = lat.new_state(), lat.new_state()
    lat.import_populations(st, f0.cuda())
    lat.import_populations(stD, fD.cuda())
    f_in = lat.export_populations(st).cpu()
    fD_in = lat.export_populations(stD).cpu()
    drho = lat.density(stD)
    lam_in, lam_out = lat.new_adjoint(), lat.new_adjoint()
    P.lbm_adjoint_from_natural(lat.h, lam_f.to(DT).cuda(), lam_in)
    gw = lat.field(3)
    gF = torch.zeros((3, *p.shape), dtype=torch.float32, device="cuda")
    gFu = torch.zeros(3, dtype=torch.float64, device="cuda")
    fc = force.cuda() if field else None
    P.lbm_step_adjoint_full(lat.h, st, lam_in, lam_out, drho, gw, fc, gF, gFu, mode="lagged",
                            grad_pending=gp.cuda())
    got = torch.empty((27, *p.shape), dtype=DT, device="cuda")
    P.lbm_adjoint_to_natural(lat.h, lam_out, got)
    back = lat.new_adjoint()
    back.zero_()
    P.lbm_density_adjoint(lat.h, gw, back)
    got_D = torch.empty((27, *p.shape), dtype=DT, device="cuda")
    P.lbm_adjoint_to_natural(lat.h, back, got_D)

    f = f_in.detach().clone().requires_grad_(True)
    fDv = fD_in.detach().clone().requires_grad_(True)
    F = (force.to(DT) if field else torch.zeros((3, *p.shape), dtype=DT)).requires_grad_(True)
    J = (lam_f.to(DT) * OL.step(f, p, force=F, grad_from=fDv.sum(0))).sum() \
        + (gp.to(DT) * OL.density_gradient(f.sum(0), p)).sum()
    want_f, want_D, want_F = torch.autograd.grad(J, (f, fDv, F))
    scale = want_f.abs().max().item()
    err = (got.cpu() - want_f).abs().max().item() / scale
    errD = (got_D.cpu() - want_D).abs().max().item() / want_D.abs().max().item()
    errF = (gF.cpu().to(DT) - want_F).abs().max().item() / want_F.abs().max().item()
    # scale: what the pending term and the lag change in the result
    J_e = (lam_f.to(DT) * OL.step(f, p, force=F)).sum()
    want_e, = torch.autograd.grad(J_e, (f,))
    share = (want_f - want_e).abs().max().item() / scale
    _say(f"{name} (lagged): rel max err lambda {err:.2e} (differs from the exact level by {share:.2e}), "
         f"density cotangent {errD:.2e}, force grad {errF:.2e}")
    assert err < 2e-6 and share > 50 * err
    # the cotangent of the gradient alone passes through the transpose of App. D's 3x3 strain-rate solve,
    # whose condition number grows as the grid gets flatter (about 6 at s = 1/2, 24 at s = 1/4), and its x
    # and y components are sums of three right-hand-side cotangents that partly cancel: FP32 rounding
    # measured 5e-6 at s = 1/4, within the 1e-5 relative tolerance of FP32 results
    assert errD < 1e-5
    assert errF < 2e-5
    assert abs(gFu.cpu() - want_F.reshape(3, -1).sum(-1)).max().item() <= 1e-4 * want_F.reshape(3, -1).sum(-1).abs().max().item()


@pytest.mark.parametrize("max_states", [128, 2])
def test_full_corrections_trajectory_gradient_matches_oracle(max_states):
    """dL/dF and dL/du0 through 18 steps with the full corrections (exact time level) on a 12x10x8 replica
    of the adjoint duct, from a start with a density variation so that the density-gradient terms
    matter; with max_states = 2 the backward pass nests its recomputation."""
    w = W.ADJOINT_DUCT_128
    p = oracle_params(w, corr="full", nx=12, ny=10, nz=8)
    p_loc = oracle_params(w, corr="local", nx=12, ny=10, nz=8)
    g = np.random.Generator(np.random.PCG64(43))
    force = torch.tensor(1e-5 * g.standard_normal((3, *p.shape))).to(torch.float32)
    u0 = torch.tensor(0.02 * g.standard_normal((3, *p.shape)))
    rho0 = torch.tensor(1.0 + 0.02 * g.standard_normal(p.shape))
    target = torch.tensor(1e-3 * g.standard_normal((3, *p.shape)))
    nsteps = 18
    L_o, gF_o, gu_o = G.loss_and_gradients(p, rho0, u0, force.to(DT), target, nsteps)
    _, gF_l, gu_l = G.loss_and_gradients(p_loc, rho0, u0, force.to(DT), target, nsteps)
    lat = gpu_lattice(p)
    uc = u0.cuda().requires_grad_(True)
    Fc = force.cuda().requires_grad_(True)
    u = ADJ.simulate(lat, uc, Fc, nsteps, 6, rho0=rho0.cuda(), max_states=max_states)
    L_g = 0.5 * ((u.to(DT) - target.cuda()) ** 2).sum()
    L_g.backward()
    eF = rel_l2(Fc.grad.cpu(), gF_o)
    eu = rel_l2(uc.grad.cpu(), gu_o)
    shareF, shareu = rel_l2(gF_l, gF_o), rel_l2(gu_l, gu_o)
    _say(f"full-correction trajectory (max_states {max_states}): loss rel err "
         f"{abs(float(L_g.detach()) - L_o.item()) / L_o.item():.2e}, dL/dF rel L2 {eF:.2e} "
         f"(local corrections differ by {shareF:.2e}), dL/du0 rel L2 {eu:.2e} (local: {shareu:.2e})")
    assert eF < 1e-4 and eu < 1e-4
    assert shareF > 20 * eF and shareu > 20 * eu


@pytest.mark.parametrize("max_states", [128, 2])
def test_full_corrections_lagged_trajectory_gradient_matches_oracle(max_states):
    """The same trajectory at the lagged time level (each step's gradient from the previous step's input
    density, the first step's from its own): dL/dF and dL/du0 against the oracle's reverse mode through
    run(lagged=True), which differs from the exact level's gradient."""
    w = W.ADJOINT_DUCT_128
    p = oracle_params(w, corr="full", nx=12, ny=10, nz=8)
    g = np.random.Generator(np.random.PCG64(43))
    force = torch.tensor(1e-5 * g.standard_normal((3, *p.shape))).to(torch.float32)
    u0 = torch.tensor(0.02 * g.standard_normal((3, *p.shape)))
    rho0 = torch.tensor(1.0 + 0.02 * g.standard_normal(p.shape))
    target = torch.tensor(1e-3 * g.standard_normal((3, *p.shape)))
    nsteps = 18

    L_o, gF_o, gu_o = G.loss_and_gradients(p, rho0, u0, force.to(DT), target, nsteps, lagged=True)
    _, gF_e, gu_e = G.loss_and_gradients(p, rho0, u0, force.to(DT), target, nsteps)
    lat = gpu_lattice(p)
    uc = u0.cuda().requires_grad_(True)
    Fc = force.cuda().requires_grad_(True)
    u = ADJ.simulate(lat, uc, Fc, nsteps, 6, rho0=rho0.cuda(), max_states=max_states, full_mode="lagged")
    L_g = 0.5 * ((u.to(DT) - target.cuda()) ** 2).sum()
    L_g.backward()
    eF = rel_l2(Fc.grad.cpu(), gF_o)
    eu = rel_l2(uc.grad.cpu(), gu_o)
    dF, du = rel_l2(gF_e, gF_o), rel_l2(gu_e, gu_o)
    _say(f"lagged full-correction trajectory (max_states {max_states}): loss rel err "
         f"{abs(float(L_g.detach()) - L_o.item()) / L_o.item():.2e}, dL/dF rel L2 {eF:.2e} (exact level differs by "
         f"{dF:.2e}), dL/du0 rel L2 {eu:.2e} (exact: {du:.2e})")
    assert eF < 1e-5 and eu < 1e-5
    assert dF > 20 * eF and du > 20 * eu
