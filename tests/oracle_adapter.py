"""Build oracle objects from the shared workload definitions (tests only)."""
from oracle.fe import Mesh
from oracle.problems import Problem


def oracle_problem(wl, **over):
    kw = dict(amp=wl.amp, p_bg=wl.p_bg, energy=wl.energy)
    kw.update(over)
    mesh = Mesh(wl.dim, tuple(wl.nel[: wl.dim]), tuple(wl.lo[: wl.dim]), tuple(wl.hi[: wl.dim]))
    return Problem(wl.problem, mesh, wl.gamma, wl.use_av, wl.cfl, **kw)
