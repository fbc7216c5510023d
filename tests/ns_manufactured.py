"""A manufactured solution of the incompressible Navier-Stokes equations on the unit cube
with no-slip walls, for the projection-step tests.

    u = g(t) sin(pi z) (d phi/dy, -d phi/dx, 0),  phi = sin^2(pi x) sin^2(pi y),
    g(t) = A (1 + sin(w t)),   p = cos(w t) cos(pi x) cos(pi y) cos(pi z),

u is divergence-free and vanishes on the six faces, p has zero mean, and the forcing is
f = du/dt - nu Lap u + (u . grad) u + grad p.  The derivatives are taken symbolically
(sympy), so no hand-derived formula enters the forcing; the divergence of u is checked
symbolically too.  The normal component of curl curl u is not zero on the faces x = 0, 1
and y = 0, 1, so the rotational term of the pressure boundary condition matters, and
(u . grad) u is of the size of the other terms.
"""
import numpy as np
import sympy as sp


def fields(nu, amp=0.5, omega=6.0):
    """(u, p, f) as functions of (x, y, z, t) on numpy arrays; u and f return 3 arrays."""
    x, y, z, t = sp.symbols("x y z t")
    X = (x, y, z)
    g = amp * (1 + sp.sin(omega * t))
    phi = sp.sin(sp.pi * x) ** 2 * sp.sin(sp.pi * y) ** 2
    h = sp.sin(sp.pi * z)
    u = [g * h * sp.diff(phi, y), -g * h * sp.diff(phi, x), sp.Integer(0)]
    p = sp.cos(omega * t) * sp.cos(sp.pi * x) * sp.cos(sp.pi * y) * sp.cos(sp.pi * z)
    assert sp.simplify(sum(sp.diff(u[i], X[i]) for i in range(3))) == 0
    f = [sp.diff(u[i], t) - nu * sum(sp.diff(u[i], X[j], 2) for j in range(3))
         + sum(u[j] * sp.diff(u[i], X[j]) for j in range(3)) + sp.diff(p, X[i]) for i in range(3)]
    lam = [sp.lambdify((x, y, z, t), e, "numpy") for e in (*u, p, *f)]

    def vec(fs):
        def ev(xyz, tt):
            return np.stack([np.broadcast_to(fc(xyz[:, 0], xyz[:, 1], xyz[:, 2], tt), (len(xyz),))
                             for fc in fs]).astype(np.float64)
        return ev

    def scal(xyz, tt):
        return np.broadcast_to(lam[3](xyz[:, 0], xyz[:, 1], xyz[:, 2], tt), (len(xyz),)).astype(np.float64)
    return vec(lam[:3]), scal, vec(lam[4:])


def run(make_stepper, xyz, m1, nu, T, nsteps, amp=0.5, omega=6.0, step=None):
    """Run nsteps steps of size T / nsteps from the exact u(0) with the nodal forcing
    f(t_{n+1}); return the relative errors of u and p (p against the exact pressure
    shifted to m1^T p = 0, the stepper's mean-zero condition) at t = T, and the fields.
    make_stepper(dt) builds the stepper; step(st, u, f) advances it (default st.step)."""
    U, P, F = fields(nu, amp, omega)
    st = make_stepper(T / nsteps)
    step = step or (lambda s, u, f: s.step(u, f))
    u = U(xyz, 0.0)
    for n in range(nsteps):
        u, p = step(st, u, F(xyz, (n + 1) * T / nsteps))
    ue = U(xyz, T)
    pe = P(xyz, T)
    pe = pe - (m1 @ pe) / m1.sum()
    eu = np.linalg.norm(u - ue) / np.linalg.norm(ue)
    ep = np.linalg.norm(p - pe) / np.linalg.norm(pe)
    return eu, ep, u, p
