"""Parameters of one oracle run (test infrastructure only)."""

from dataclasses import dataclass

# Correction variants of the extended equilibria (Sec. 2.4 / App. D):
#   "off"     -- plain central-moment collision, no cuboid corrections
#   "lowmach" -- theta without the 3u^2 terms, lambda = 0 (last remark of Sec. 2.4)
#   "local"   -- theta with the 3u^2 terms, lambda = 0 (density-gradient terms dropped)
#   "full"    -- theta and lambda; needs the density gradient from a finite-difference stencil
CORRECTIONS = ("off", "lowmach", "local", "full")
BOUNDARIES = ("periodic", "bounceback")
# Moments relaxed by the collision: "central" (3DCCM-LBM, Sec. 3.2) or "raw"
# (3DCRM-LBM: the same steps without the frame transformations, Sec. 3.1 and Sec. 7)
MOMENT_BASES = ("central", "raw")


@dataclass(frozen=True)
class Params:
    nx: int
    ny: int
    nz: int
    r: float = 1.0            # grid aspect ratio dy/dx (Sec. 2.1)
    s: float = 1.0            # grid aspect ratio dz/dx (Sec. 2.1)
    cs2: float = 0.0          # squared sound speed; <= 0 selects min(r^2, s^2)/3 (end of Sec. 2.5)
    omega_nu: float = 1.0     # shear rate: k_110, k_101, k_011, k_2d1, k_2d2 (App. D)
    omega_xi: float = 1.0     # bulk rate: trace k_2s (App. D)
    omega_1: float = 1.0      # first-order rate (has no effect, see App. D)
    omega_hi: float = 1.0     # every third- and higher-order rate (1 in the paper)
    corr: str = "local"
    bc_y: str = "periodic"
    bc_z: str = "periodic"
    bc_x: str = "periodic"
    # tangential velocity of each wall face, in the order x-, x+, y-, y+, z-, z+
    # (used on bounce-back axes only; Sec. 4, momentum-augmented bounce-back)
    wall_velocity: tuple = ((0.0, 0.0, 0.0),) * 6
    moments: str = "central"

    def __post_init__(self):
        assert self.corr in CORRECTIONS, self.corr
        assert self.moments in MOMENT_BASES, self.moments
        assert self.bc_x in BOUNDARIES and self.bc_y in BOUNDARIES and self.bc_z in BOUNDARIES
        wv = tuple(tuple(float(c) for c in v) for v in self.wall_velocity)
        assert len(wv) == 6 and all(len(v) == 3 for v in wv)
        for face, v in enumerate(wv):
            assert v[face // 2] == 0.0, "a wall moves only tangentially"
        object.__setattr__(self, "wall_velocity", wv)
        if self.cs2 <= 0.0:
            object.__setattr__(self, "cs2", min(self.r ** 2, self.s ** 2) / 3.0)

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)
