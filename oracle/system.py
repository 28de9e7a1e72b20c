"""The assembled micromagnetic problem (FP64 oracle).

For each magnet the paper integrates dm/dt = tau (Eq. 1), tau = LLG torque
(Eq. 2) plus spin-transfer torque, with the effective field summed from the
terms in ``fields``/``demag`` (Methods, "Micromagnetism").  A magnet of two
or three sublattices couples them through Eq. 3 (for three, every pair with
the same A12 and A0: B^(s) gains sum over s' != s of A12/Ms lap m^(s') +
4 A0/(Ms a^2) m^(s'), the paper's three exchange-coupled sublattices of the
non-collinear Mn3Sn demonstration) and shares one demagnetising field built
from the summed moment.  In a polycrystalline magnet (grain ids per cell)
the A11 and A12 stencil links between cells of different grains carry
grain_exchange_scale times the constant (the paper's domain-wall mobility
and Mn3Sn demonstrations reduce both at grain boundaries).  With elasticity on, the displacement u
and velocity v join the state (Eq. 7) and the strain feeds Eq. 9 back.

Energies (joules, FP64) follow one rule for every term bilinear in m:
E = -1/2 sum_s Ms^(s) m^(s) . B_term^(s) V per cell; Zeeman is
-sum_s Ms m.B_ext V, uniaxial -Ku1 (u.m)^2 - Ku2 (u.m)^4, cubic
Kc1 (a1^2 a2^2 + a2^2 a3^2 + a3^2 a1^2), magnetoelastic
sum_s [B1 sum_i eps_ii m_i^2 + 2 B2 sum_{i<j} eps_ij m_i m_j], elastic
1/2 sigma:eps + 1/2 rho v^2 (all per unit volume, times V).
"""
from __future__ import annotations

import numpy as np

from . import elastic as el
from . import fields as fl
from . import dmi
from . import torque as tq
from .demag import Demag
from .rk import FAC_MAX, FAC_MIN, SAFETY, TABLEAUS, Stepper, new_dt

TERMS = ("demag", "exch", "afm_nn", "afm_cell", "dmi", "anis_u", "anis_c",
         "zeeman", "mel")


class Problem:
    def __init__(self, p, N6=None, demag_workers=None):
        self.p = p
        self.n = tuple(p["n"])
        self.d = tuple(p["cell"])
        self.nsub = p["nsub"]
        self.V = self.d[0] * self.d[1] * self.d[2]
        if p["nsub"] >= 2 and any(v != 0.0 for v in p["Dint"]):
            raise ValueError("interfacial DMI is implemented for one sublattice")
        if p["nsub"] == 3 and (p.get("bc", "open") == "eq6" or p["elastic"] is not None
                               or any(p.get("dmi_homo", (0, 0, 0)))):
            raise ValueError("three sublattices: open boundaries, no elasticity, no "
                             "homogeneous DMI")
        # periodic boundaries: image repetitions per axis (0 = open)
        self.pbc = tuple(int(v) for v in p.get("pbc", (0, 0, 0)))
        if any(v < 0 for v in self.pbc) or self.pbc[2] != 0:
            raise ValueError("periodic boundaries are supported along x and y")
        if any(self.pbc) and p["elastic"] is not None:
            raise ValueError("periodic boundaries are not combined with elasticity")
        self.periodic = tuple(v > 0 for v in self.pbc)
        # exchange scale at grain boundaries (1 = none)
        gscale = p.get("grain_exchange_scale", 1.0)
        self.links = None
        if p.get("grain") is not None and gscale != 1.0:
            self.links = fl.link_weights(p["grain"], gscale, self.periodic)
        # boundary condition of the stencils: "open" (ghost = boundary cell,
        # or the Eq. 5 ghosts of the interfacial DMI) or "eq6" (Eq. 6 with
        # the general DMI tensors of Eq. 4)
        self.eq6 = p.get("bc", "open") == "eq6"
        W, W12 = p.get("dmi_W"), p.get("dmi_W12")
        self.W = np.zeros((self.nsub, 3, 3)) if W is None else np.asarray(W, dtype=np.float64)
        self.W12 = np.zeros((3, 3)) if W12 is None else np.asarray(W12, dtype=np.float64)
        if (np.any(self.W) or np.any(self.W12)) and not self.eq6:
            raise ValueError("DMI tensors need the Eq. 6 boundary condition (bc='eq6')")
        if self.eq6 and any(v != 0.0 for v in p["Dint"]):
            raise ValueError("with bc='eq6' give the interfacial DMI as a tensor")
        self.demag = Demag(self.n, self.d, N6, demag_workers, self.pbc) if p["demag"] else None
        self.axis = None
        if p.get("grain") is not None:
            self.axis = np.moveaxis(np.asarray(p["grain_axes"])[p["grain"]], -1, 0)
        self.tableau = TABLEAUS[p.get("solver", "dp45")]
        self.stepper = Stepper(self.rhs, self.normalise, self.err_norm, self.tableau)

    # ----------------------------------------------------------- fields --
    def strain(self, u):
        return el.strain(u, self.d)

    def term_field(self, name, m, s, u=None, Bd=None):
        p, d = self.p, self.d
        ms = m[s]
        Ms = p["Ms"][s]
        # the other sublattices (Eq. 3 with one A12 and one A0 for every pair)
        others = [m[o] for o in range(self.nsub) if o != s]
        other = others[0] if self.nsub == 2 else None
        if name == "demag":
            if self.demag is None:
                return np.zeros_like(ms)
            if Bd is None:
                Bd = self.demag_field(m)
            return Bd.copy() if Ms != 0.0 else np.zeros_like(ms)
        if self.eq6 and name in ("exch", "afm_nn", "dmi"):
            return self._eq6_term(name, m, s)
        if name == "exch":
            return fl.exchange_field(ms, Ms, p["A11"][s], d, p["Dint"][s],
                                     p["dmi_layer"], self.periodic, self.links)
        if name == "afm_nn":
            B = np.zeros_like(ms)
            for mo in others:
                B = B + fl.afm_nn_field(mo, Ms, p["A12"], d, self.periodic, self.links)
            return B
        if name == "afm_cell":
            B = np.zeros_like(ms)
            for mo in others:
                B = B + fl.afm_cell_field(mo, Ms, p["A0"], p["latcon"])
            return B
        if name == "dmi":
            B = fl.dmi_field(ms, Ms, p["A11"][s], p["Dint"][s], d,
                             p["dmi_layer"], self.periodic)
            if other is not None:
                B = B + fl.homogeneous_dmi_field(ms, other, Ms, p.get("dmi_homo", (0, 0, 0)),
                                                 s == 0)
            return B
        if name == "anis_u":
            ax = self.axis if self.axis is not None else p["anis_u"][s]
            return fl.uniaxial_field(ms, Ms, p["Ku1"][s], p["Ku2"][s], ax)
        if name == "anis_c":
            return fl.cubic_field(ms, Ms, p["Kc1"][s], p["cub_c1"][s], p["cub_c2"][s])
        if name == "zeeman":
            return fl.zeeman_field(ms, p["B_ext"])
        if name == "mel":
            if p["elastic"] is None or u is None:
                return np.zeros_like(ms)
            return fl.magnetoelastic_field(ms, Ms, p["B1"][s], p["B2"][s],
                                           self.strain(u))
        raise KeyError(name)

    def _lap(self, g):
        if self.links is None:
            return fl.laplacian(g, self.d)
        return fl.laplacian_weighted(g, self.d, self.links)

    def _eq6_term(self, name, m, s):
        """Exchange, inter-sublattice exchange or DMI over the Eq. 6 ghosts."""
        p, d = self.p, self.d
        Ms = p["Ms"][s]
        if Ms == 0.0:
            return np.zeros_like(m[s])
        g = dmi.eq6_ghosts(np.asarray(m), d, p["A11"], p["A12"], self.W, self.periodic)
        o = 1 - s if self.nsub == 2 else None
        if name == "exch":
            return (2.0 * p["A11"][s] / Ms) * self._lap(g[s])
        if name == "afm_nn":
            if o is None:
                return np.zeros_like(m[s])
            return (p["A12"] / Ms) * self._lap(g[o])
        B = dmi.tensor_field(g[s], None if o is None else g[o], Ms, self.W[s], self.W12, d)
        if o is not None:
            B = B + fl.homogeneous_dmi_field(m[s], m[o], Ms, p.get("dmi_homo", (0, 0, 0)),
                                             s == 0)
        return B

    def demag_field(self, m):
        M = sum(self.p["Ms"][s] * m[s] for s in range(self.nsub))
        return self.demag.field(M)

    def eval_heff(self, m, terms=TERMS, u=None):
        """Sum of the named terms, shape (nsub, 3, nz, ny, nx)."""
        Bd = self.demag_field(m) if (self.demag is not None and "demag" in terms) else None
        out = np.zeros_like(m, dtype=np.float64)
        for s in range(self.nsub):
            for name in terms:
                out[s] += self.term_field(name, m, s, u, Bd)
        return out

    # --------------------------------------------------------- energies --
    def energies(self, m, u=None, v=None, t=0.0):
        p, V = self.p, self.V
        E = {}
        Bd = self.demag_field(m) if self.demag is not None else None
        for name in ("demag", "exch", "afm_nn", "afm_cell", "dmi"):
            acc = 0.0
            for s in range(self.nsub):
                B = self.term_field(name, m, s, u, Bd)
                acc += -0.5 * p["Ms"][s] * np.sum(m[s] * B)
            E[name] = acc * V
        acc = 0.0
        for s in range(self.nsub):
            ax = self.axis if self.axis is not None else p["anis_u"][s]
            ax = np.asarray(ax, dtype=np.float64)
            if ax.ndim == 1:
                ax = ax[:, None, None, None]
            um = np.sum(ax * m[s], axis=0)
            if p["Ms"][s] != 0.0:
                acc += np.sum(-p["Ku1"][s] * um ** 2 - p["Ku2"][s] * um ** 4)
        E["anis_u"] = acc * V
        acc = 0.0
        for s in range(self.nsub):
            if p["Ms"][s] == 0.0:
                continue
            cs = fl.cubic_frame(p["cub_c1"][s], p["cub_c2"][s])
            a = [np.tensordot(c, m[s], axes=(0, 0)) for c in cs]
            acc += p["Kc1"][s] * np.sum(a[0] ** 2 * a[1] ** 2 + a[1] ** 2 * a[2] ** 2
                                        + a[2] ** 2 * a[0] ** 2)
        E["anis_c"] = acc * V
        acc = 0.0
        for s in range(self.nsub):
            Bz = np.asarray(p["B_ext"], dtype=np.float64)[:, None, None, None]
            acc += -p["Ms"][s] * np.sum(m[s] * Bz)
        E["zeeman"] = acc * V
        acc = 0.0
        if p["elastic"] is not None and u is not None:
            eps = self.strain(u)
            for s in range(self.nsub):
                if p["Ms"][s] == 0.0:
                    continue
                mm = m[s]
                B1, B2 = p["B1"][s], p["B2"][s]
                acc += np.sum(B1 * (eps[0] * mm[0] ** 2 + eps[1] * mm[1] ** 2
                                    + eps[2] * mm[2] ** 2)
                              + 2.0 * B2 * (eps[3] * mm[0] * mm[1] + eps[4] * mm[0] * mm[2]
                                            + eps[5] * mm[1] * mm[2]))
        E["mel"] = acc * V
        if p["elastic"] is not None and u is not None:
            vv = np.zeros_like(u) if v is None else v
            E["elastic"] = np.sum(el.elastic_energy_density(u, vv, self.d, p["elastic"])) * V
        else:
            E["elastic"] = 0.0
        return E

    # ------------------------------------------------------------ dynamics
    def torque(self, m, u=None):
        p = self.p
        B = self.eval_heff(m, TERMS, u)
        out = np.empty_like(m)
        for s in range(self.nsub):
            out[s] = tq.llg_torque(m[s], B[s], p["gamma"], p["alpha"][s])
            uu = tq.drift_velocity(p["zl_P"][s], p["j"], p["Ms"][s])
            if np.any(uu):
                out[s] += tq.zhang_li_torque(m[s], uu, p["alpha"][s], p["zl_xi"][s], self.d,
                                             self.periodic)
        return out

    def rhs(self, t, y):
        m = y[0]
        if self.p["elastic"] is None:
            return [self.torque(m)]
        u, v = y[1], y[2]
        e = self.p["elastic"]
        f = el.elastic_force(u, self.d, self.n, t, e, v)
        for s in range(self.nsub):
            if self.p["Ms"][s] != 0.0:
                f = f + el.magnetoelastic_force(m[s], self.p["B1"][s], self.p["B2"][s], self.d)
        dv = (f - e["eta"] * v) / e["rho"]
        return [self.torque(m, u), v.copy(), dv]

    @staticmethod
    def normalise(y):
        out = list(y)
        out[0] = y[0] / np.linalg.norm(y[0], axis=1, keepdims=True)
        return out

    @staticmethod
    def err_norm(errv):
        return float(np.max(np.linalg.norm(errv[0], axis=1)))

    def initial_state(self, m):
        y = [np.asarray(m, dtype=np.float64).copy()]
        if self.p["elastic"] is not None:
            y.append(np.zeros((3,) + self.n[::-1]))
            y.append(np.zeros((3,) + self.n[::-1]))
        return y

    def run_fixed(self, y, t0, dt, nsteps):
        """nsteps steps of size dt with no step control."""
        t = t0
        for i in range(nsteps):
            y, knext, _ = self.stepper.step(t, y, dt)
            self.stepper.accept(knext)
            t = t0 + (i + 1) * dt
        return y, t

    def run(self, y, t0, t_end, tol=1e-5, dt0=1e-14, dt_min=1e-20,
            sample_every=None, sample=None, max_steps=10 ** 9):
        """Adaptive stepping from t0 to t_end; returns (y, t, info, samples).

        A step that would pass the next output time (t0 + k*sample_every,
        or t_end) is shortened to land on it exactly.  An output time closer
        to t_end than 1e-9 of the run length is t_end itself: k*sample_every
        can fall a few ulp short of t_end, and landing on both would take a
        step of ~1e-26 s that the step-size floor rejects.
        """
        t = t0
        p = self.p
        ctl = dict(safety=p.get("safety") or SAFETY, fac_min=p.get("fac_min") or FAC_MIN,
                   fac_max=p.get("fac_max") or FAC_MAX, dt_max=p.get("dt_max") or None)
        if not (0.0 < ctl["fac_min"] < 1.0 and 0.0 < ctl["safety"] <= 1.0
                and ctl["fac_max"] >= 1.0):
            # a rejected attempt must shrink the step, or the loop never ends
            raise ValueError("step control: fac_min in (0, 1), safety in (0, 1], fac_max >= 1")
        dt = dt0 if not ctl["dt_max"] else min(dt0, ctl["dt_max"])
        samples = [] if sample is None else [(t, sample(y))]
        k = 1

        def out_time(k):
            o = t0 + k * sample_every
            return t_end if o >= t_end - 1e-9 * (t_end - t0) else o

        next_out = out_time(1) if sample_every else t_end
        steps = rejects = 0
        while t < t_end and steps + rejects < max_steps:
            target = min(next_out, t_end)
            remaining = target - t
            land = dt >= remaining
            h = remaining if land else dt
            ynew, knext, err = self.stepper.step(t, y, h)
            if err <= tol:
                y = ynew
                self.stepper.accept(knext)
                t = target if land else t + h
                steps += 1
                if land and sample_every and t == next_out:
                    if sample is not None:
                        samples.append((t, sample(y)))
                    k += 1
                    next_out = out_time(k)
            else:
                rejects += 1
            dt = new_dt(h, err, tol, self.tableau.q, **ctl)
            if dt < dt_min:
                raise RuntimeError("time step underflow")
        return y, t, dict(steps=steps, rejects=rejects, dt=dt), samples
