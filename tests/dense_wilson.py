"""Dense Wilson hopping matrix on tiny lattices, assembled site by site.

Used as an independent check of the oracle's field-based hopping term: this
builds the 12V x 12V matrix from explicit loops over sites and directions,
placing spin-projector (x) colour-link blocks at (row site, column site).
On a lattice with L_mu = 2 the forward and backward neighbours in direction
mu coincide and both blocks are added to the same position.

Vector index = site * 12 + spin * 3 + colour, site = ((t Lz + z) Ly + y) Lx + x.
"""

import numpy as np

from oracle.dirac import GAMMA, ONE4


def site_index(c, dims):
    x, y, z, t = c
    lx, ly, lz, lt = dims
    return ((t * lz + z) * ly + y) * lx + x


def dense_dhop(U, dims, bc=(1, 1, 1, -1), dagger=False):
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    sg = -1.0 if dagger else 1.0
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    c = [x, y, z, t]
                    row = site_index(c, dims)
                    for mu in range(4):
                        up = list(c)
                        up[mu] = (c[mu] + 1) % dims[mu]
                        s_up = bc[mu] if c[mu] == dims[mu] - 1 else 1
                        dn = list(c)
                        dn[mu] = (c[mu] - 1) % dims[mu]
                        s_dn = bc[mu] if c[mu] == 0 else 1
                        u_here = U[t, z, y, x, mu]
                        u_dn = U[dn[3], dn[2], dn[1], dn[0], mu]
                        cu = site_index(up, dims)
                        cd = site_index(dn, dims)
                        D[12 * row:12 * row + 12, 12 * cu:12 * cu + 12] += \
                            s_up * np.kron(ONE4 - sg * GAMMA[mu], u_here)
                        D[12 * row:12 * row + 12, 12 * cd:12 * cd + 12] += \
                            s_dn * np.kron(ONE4 + sg * GAMMA[mu], u_dn.conj().T)
    return D


def parity_vector(dims):
    lx, ly, lz, lt = dims
    par = np.zeros(lx * ly * lz * lt, dtype=int)
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    par[site_index([x, y, z, t], dims)] = (x + y + z + t) % 2
    return np.repeat(par, 12)
