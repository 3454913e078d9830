"""Differentiable trajectories of the cuboid LB step (torch.autograd.Function).

``simulate(lat, u0, force, nsteps, checkpoint_every)`` runs
    f(0) = f_eq(rho0, u0);  nsteps collide-and-stream steps under a per-node
    body force (or the lattice's uniform force);  u(T) from eq. 12
and returns u(T) as a differentiable tensor.  Its backward pass runs the
hand-written adjoint kernels of the library: lbm_moments_adjoint for the
observables, lbm_step_adjoint once per step in reverse order, and
lbm_init_adjoint for the initial velocity; the force gradient accumulates
inside the adjoint step kernel.  With the full corrections the trajectory
steps at the exact (default) or the lagged time level of the density gradient
(lbm_step_full) and reverses through lbm_step_adjoint_full; at the lagged level
the cotangent of each step's gradient belongs to the state one step earlier, so
it is handed to the next call of the sweep, and the first step's (taken from
its own input) goes to lambda(0) through lbm_density_adjoint; at the exact
level the recomputed steps keep the density of each state they step from, so
its adjoint step reads it instead of computing it again.

Memory: the forward keeps one state every ``checkpoint_every`` steps; the
backward recomputes one segment at a time from its checkpoint, holding that
segment's states while it steps back through it.  A segment longer than
``max_states`` is split again: its sub-segment starts (about sqrt(K) of
them) are recomputed and kept, then each sub-segment is recomputed and
reversed in turn (one extra forward pass per segment).  Peak memory is about
nsteps/K + min(K, 2 sqrt(K)) states plus two adjoint buffers (with the full
corrections also one density field, 4 B per node, per held state).
"""

import math

import torch

from . import _lib
from . import lbm as L


class _Steps:
    """Forward and adjoint steps of a lattice: plain, or with the full corrections at the exact or the
    lagged time level of the density gradient (whose fields this holds).  ``dens`` is a density field
    that a state's adjoint step reads: at the lagged level the one its step took the gradient from, at
    the exact level the state's own density where a recomputed step already wrote it (else None)."""

    def __init__(self, lat, mode):
        self.lat = lat
        self.full = lat.h.params.corr == _lib.CORR["full"]
        self.lagged = self.full and mode == "lagged"
        self.drho = lat.field(1) if self.full and not self.lagged else None
        self.grad = self.pending = None

    def start(self, a):
        """The density field of the first step from state a (lagged level: a's own density)."""
        return self.lat.density(a) if self.lagged else None

    def advance(self, a, b, n, force, dens):
        """n steps; returns (current, scratch, density field of the next step)."""
        if self.lagged:
            other = self.lat.field(1)
            a, b, dens, _ = self.lat.step_full(a, b, n, dens, other, "lagged", force)
            return a, b, dens
        if self.full:
            a, b, _, _ = self.lat.step_full(a, b, n, self.drho, None, "exact", force)
            return a, b, None
        a, b = self.lat.step(a, b, n, force)
        return a, b, None

    def recompute(self, states, start_dens, force):
        """Step states[0] -> states[1] -> ... (each from the one before); returns for each state the
        density field its adjoint step reads: lagged level, the field its step took the gradient from
        (start_dens for the first); exact level, its own density as its step computed it (None for the
        last state, which is not stepped from here: its adjoint step computes it)."""
        h, n = self.lat.h, len(states)
        if self.lagged:
            dens = [start_dens]
            for i in range(1, n):
                nxt = self.lat.field(1)
                L.lbm_step_full(h, 1, states[i - 1], states[i], dens[i - 1], nxt, "lagged", force)
                dens.append(nxt)
            return dens
        if self.full:
            dens = []
            for i in range(1, n):
                d = self.lat.field(1)
                L.lbm_step_full(h, 1, states[i - 1], states[i], d, None, "exact", force)
                dens.append(d)
            return dens + [None]
        for i in range(1, n):
            L.lbm_step(h, 1, states[i - 1], states[i], force)
        return [None] * n

    def adjoint(self, state, dens, lam, lam_next, force, grad_force):
        if not self.full:
            L.lbm_step_adjoint(self.lat.h, state, lam, lam_next, force, grad_force)
            return
        if self.grad is None:
            self.grad = self.lat.field(3)
        if not self.lagged:
            if dens is None:    # the density pass runs inside the call
                L.lbm_step_adjoint_full(self.lat.h, state, lam, lam_next, self.drho, self.grad, force, grad_force)
            else:               # the recomputed step from this state already wrote its density
                L.lbm_step_adjoint_full(self.lat.h, state, lam, lam_next, dens, self.grad, force, grad_force,
                                        mode="exact_drho")
            return
        # lagged: the cotangent of this step's gradient belongs to the state before it (the pending
        # transpose is added to that state's adjoint by the next call of the sweep)
        L.lbm_step_adjoint_full(self.lat.h, state, lam, lam_next, dens, self.grad, force, grad_force, mode="lagged",
                                grad_pending=self.pending)
        if self.pending is None:
            self.pending = self.lat.field(3)
        self.grad, self.pending = self.pending, self.grad

    def finish(self, lam0):
        """After the sweep: the first step's gradient came from the initial state's own density."""
        if self.lagged and self.pending is not None:
            L.lbm_density_adjoint(self.lat.h, self.pending, lam0)


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, force, lat, rho0, nsteps, every, max_states, full_mode):
        force_t = force if force.numel() else None
        steps = _Steps(lat, full_mode)
        a, b = lat.new_state(), lat.new_state()
        lat.init(a, rho=rho0, u=u0)
        dens = steps.start(a)
        # each checkpoint keeps the handle's step counter too, so that a recomputed segment
        # rounds exactly like the forward pass (stochastic rounding of BF16-SR storage), and at the
        # lagged time level the density field its first step takes the gradient from
        checkpoints, counters = [a.clone()], [L.lbm_step_counter(lat.h)]
        dens_at = [None if dens is None else dens.clone()]
        t = 0
        while t < nsteps:
            n = min(every, nsteps - t)
            a, b, dens = steps.advance(a, b, n, force_t, dens)
            t += n
            if t < nsteps:
                checkpoints.append(a.clone())
                counters.append(L.lbm_step_counter(lat.h))
                dens_at.append(None if dens is None else dens.clone())
        m = lat.moments(a, force_t, sums=False)
        ctx.lat, ctx.nsteps, ctx.every, ctx.max_states = lat, nsteps, every, max_states
        ctx.checkpoints, ctx.counters, ctx.dens_at, ctx.final = checkpoints, counters, dens_at, a
        ctx.counter_end = L.lbm_step_counter(lat.h)
        ctx.force, ctx.rho0, ctx.steps = force_t, rho0, steps
        ctx.save_for_backward(u0)
        ctx.force_needs_grad = force.requires_grad
        return m.u

    @staticmethod
    def backward(ctx, g_u):
        lat, h = ctx.lat, ctx.lat.h
        (u0,) = ctx.saved_tensors
        force = ctx.force
        grad_force = None
        if ctx.force_needs_grad:
            grad_force = torch.zeros((3, *lat.shape), dtype=torch.float32, device=lat.device)
        lam = lat.new_adjoint(zero=False)
        lam_next = lat.new_adjoint(zero=False)
        L.lbm_moments_adjoint(h, ctx.final, lam, force=force, g_u=g_u.to(torch.float32).contiguous(),
                              grad_force=grad_force)
        ctx.final = None
        nseg = len(ctx.checkpoints)
        pool = _StatePool(lat)
        for seg in reversed(range(nseg)):
            start = seg * ctx.every
            n = min(ctx.every, ctx.nsteps - start)
            lam, lam_next = _reverse_segment(ctx.steps, ctx.checkpoints[seg], ctx.dens_at[seg], ctx.counters[seg],
                                             n, lam, lam_next, force, grad_force, ctx.max_states, pool)
            ctx.checkpoints[seg] = ctx.dens_at[seg] = None
        ctx.steps.finish(lam)
        L.lbm_set_step_counter(h, ctx.counter_end)
        g_u0 = torch.empty((3, *lat.shape), dtype=torch.float64, device=lat.device)
        rho0 = None if ctx.rho0 is None else ctx.rho0.to(torch.float64).contiguous()
        L.lbm_init_adjoint(h, lam, rho=rho0, u=u0.contiguous(), g_u=g_u0)
        return g_u0, grad_force, None, None, None, None, None, None


class _StatePool:
    """Reusable state buffers for the recomputation (allocated on first use)."""

    def __init__(self, lat):
        self.lat, self.free = lat, []

    def get(self):
        return self.free.pop() if self.free else self.lat.new_state()

    def put(self, *states):
        self.free.extend(states)


def _reverse_segment(steps, start_state, start_dens, counter, n, lam, lam_next, force, grad_force, max_states,
                     pool):
    """Apply the adjoint of n steps starting from ``start_state`` (taken with step counter ``counter``, its
    first step's gradient from ``start_dens`` at the lagged time level); returns the swapped adjoint
    buffers."""
    h = steps.lat.h
    if n <= max_states:
        states = [start_state] + [pool.get() for _ in range(n - 1)]
        L.lbm_set_step_counter(h, counter)
        dens = steps.recompute(states, start_dens, force)
        for i in reversed(range(n)):
            steps.adjoint(states[i], dens[i], lam, lam_next, force, grad_force)
            lam, lam_next = lam_next, lam
        pool.put(*states[1:])
        return lam, lam_next
    sub = max(1, math.ceil(math.sqrt(n)))
    starts, sub_dens = [], []
    cur, tmp = pool.get(), pool.get()
    cur.copy_(start_state)
    dens = start_dens
    L.lbm_set_step_counter(h, counter)
    for s0 in range(0, n, sub):
        keep = pool.get()
        keep.copy_(cur)
        starts.append(keep)
        sub_dens.append(None if dens is None else dens.clone())
        m = min(sub, n - s0)
        if s0 + m < n:
            cur, tmp, dens = steps.advance(cur, tmp, m, force, dens)
    pool.put(cur, tmp)
    for j in reversed(range(len(starts))):
        m = min(sub, n - j * sub)
        lam, lam_next = _reverse_segment(steps, starts[j], sub_dens[j], counter + j * sub, m, lam, lam_next, force,
                                         grad_force, max_states, pool)
        pool.put(starts[j])
    return lam, lam_next


def simulate(lat, u0, force=None, nsteps=1, checkpoint_every=50, rho0=None, max_states=128, full_mode="exact"):
    """u(T) after ``nsteps`` steps from f_eq(rho0, u0); differentiable in u0 and force.

    lat:   a ``Lattice``
    u0:    (3, nz, ny, nx) float64 on the lattice device
    force: (3, nz, ny, nx) float32 per-node body force, or None for the lattice's uniform force
    max_states: most states one segment may hold during the backward pass (nesting beyond)
    full_mode: with the full corrections, the time level of the density gradient ("exact" or
           "lagged", as lbm_step_full; the lagged run's first step takes its own input's density)

    Raises ValueError unless nsteps >= 0, checkpoint_every >= 1 and max_states >= 1.
    """
    if int(nsteps) < 0:
        raise ValueError(f"nsteps must be >= 0, got {nsteps}")
    if int(checkpoint_every) < 1:
        raise ValueError(f"checkpoint_every must be >= 1, got {checkpoint_every}")
    if int(max_states) < 1:
        raise ValueError(f"max_states must be >= 1, got {max_states}")
    if full_mode not in ("exact", "lagged"):
        raise ValueError(f"full_mode must be 'exact' or 'lagged', got {full_mode!r}")
    if force is None:
        force = torch.empty(0, dtype=torch.float32, device=lat.device)
    return _Trajectory.apply(u0, force, lat, rho0, int(nsteps), int(checkpoint_every), int(max_states), full_mode)


def uniform_force_gradient(lat, state_t, lam_in, lam_out, force=None):
    """One adjoint step that also returns d/dF of the uniform force (FP64 [3])."""
    g = torch.zeros(3, dtype=torch.float64, device=lat.device)
    L.lbm_step_adjoint(lat.h, state_t, lam_in, lam_out, force, None, g)
    return g
