"""Named workloads (physical parameters only).

C1  plain FP64, N_c = 150: t in [-5, 5], dt = dtau = 0.2, beta = 10, U = 0.5,
    E = 1, 10 x 10 Gauss-Hermite points, 10 iterations from Sigma = 0.
C2  plain FP64 at paper scale, N_c = 1800: t in [-10, 30], dt = dtau = 0.05,
    beta = 10, U in {0.5, 1, 1.5, 2}, E = 1, 55 x 55 points, to delta < 1e-8.
C3  mixed precision on the C1 contour: U = 1, E in {0.5, 1, 2, 4}.
C4  batched uneven sweep: 32 (U, E) instances with N_c from 500 to 1800.
C5  learned warm start: trained at N_c = 600, tested on the C2 contour.
Half filling uses the particle-hole symmetric convention (mu = 0, w1 = 1/2).
"""
import dataclasses


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    t_min: float
    t_max: float
    dt: float
    dtau: float
    beta: float
    U: float
    E: float
    n_eps: int
    n_ebar: int
    mu: float = 0.0
    w1: float = 0.5

    def contour(self):
        return dict(t_min=self.t_min, t_max=self.t_max, dt=self.dt,
                    dtau=self.dtau, beta=self.beta)

    def model(self):
        return dict(U=self.U, E=self.E, mu=self.mu, w1=self.w1,
                    n_eps=self.n_eps, n_ebar=self.n_ebar)

    def kwargs(self):
        d = self.contour()
        d.update(self.model())
        return d


C1 = Workload("C1", -5.0, 5.0, 0.2, 0.2, 10.0, 0.5, 1.0, 10, 10)
C1_ITERS = 10


def c2(U=1.0):
    return Workload(f"C2_U{U}", -10.0, 30.0, 0.05, 0.05, 10.0, U, 1.0, 55, 55)


def long_contour(U=1.0, E=1.0):
    """The paper's long runs (Figs. 7-9): t in [-5, 195], dt = dtau = 0.1,
    beta = 10, N_c = 4100, here with the C2 quadrature (55 x 55 points)."""
    return Workload(f"LONG_U{U}_E{E}", -5.0, 195.0, 0.1, 0.1, 10.0, U, E, 55, 55)


C2_U = (0.5, 1.0, 1.5, 2.0)
C2_TOL = 1e-8


def c3(E):
    return Workload(f"C3_E{E}", -5.0, 5.0, 0.2, 0.2, 10.0, 1.0, E, 10, 10)


C3_E = (0.5, 1.0, 2.0, 4.0)


def c4_instances(seed=0, count=32):
    """C4: a batched uneven sweep of `count` (U, E) instances, U ~ U[0.25, 2.5],
    E ~ U[0.5, 4], (dt, t_max) uniform on {0.1, 1/15, 0.05} x {10, 20, 30},
    t_min = -10, dtau = dt, beta = 10 (so N_c = (2 t_max + 30)/dt in
    {500 .. 1800}), Gauss-Hermite order n = 35 + round(20 (N_c - 500)/1300)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        u = float(rng.uniform(0.25, 2.5))
        e = float(rng.uniform(0.5, 4.0))
        dt = (0.1, 1.0 / 15.0, 0.05)[int(rng.integers(3))]
        t_max = (10.0, 20.0, 30.0)[int(rng.integers(3))]
        n_c = int(round((2 * t_max + 30) / dt))
        n = 35 + int(round(20 * (n_c - 500) / 1300))
        out.append(dict(t_min=-10.0, t_max=t_max, dt=dt, dtau=dt, beta=10.0, U=u, E=e,
                        n_eps=n, n_ebar=n))
    return out
