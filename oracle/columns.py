"""Column-wise boundaries for the vertical bonds (test infrastructure only).

App. C computes the horizontal terms of row k from 3-line networks between
the row's upper and lower boundary MPS, and says the vertical terms can be
computed similarly.  The default reading (``oracle.vmc``) contracts the 2-row
network of rows k and k+1.  This module is the other reading: the vertical
bond (y,x)-(y+1,x) is the horizontal bond (x,y)-(x,y+1) of the transposed
lattice (site (y,x) -> (x,y), legs (l,u,r,d) -> (u,l,d,r): the same state),
whose 3-line networks run between column boundary MPS.

* ``transposed``, ``transpose_tensors``, ``transpose_spins``, ``untranspose_spins``
  -- the transposed lattice, tensors and configurations.
* ``eval_config`` -- Psi, G and the horizontal ratios from the row networks
  (``vmc.eval_config``), the vertical ratios from the transposed lattice's
  horizontal ratios, and E_loc from all of them.
* ``run_chain``   -- a sweep visits the horizontal bonds row by row with the
  row boundaries (``vmc._top_down_pass`` without its vertical bonds), then the
  vertical bonds column by column: the transposed lattice's horizontal pass,
  with its own lower boundaries, its Philox key word 1 offset by COLUMN_KEY;
  each measured sweep is ``eval_config`` of the final configuration.

Only the nearest-neighbour model (J2 = 0) on the square geometry is covered:
the diagonal terms need the 2-row networks.
"""
from . import lattice as L
from .lattice import bonds, local_energy
from . import vmc

COLUMN_KEY = 1 << 16  # Philox key word 1 of the column pass: lattice id + COLUMN_KEY


def _check(lat):
    if lat.diagonals or lat.geometry != "square":
        raise ValueError("column-wise vertical bonds cover the nearest-neighbour square lattice only")


def transposed(lat):
    """The Lx x Ly lattice of the transposed PEPS (same D, Dc, couplings and truncation)."""
    _check(lat)
    return L.transpose_lattice(lat)


def transpose_tensors(T, lat):
    _check(lat)
    return L.transpose_tensors(T, lat)


transpose_spins = L.transpose_spins
untranspose_spins = L.untranspose_spins


def eval_config(T, lat, spins):
    """dict(sign, log_abs_psi, e_loc, dlnpsi, ratios) with the vertical ratios from column boundaries."""
    _check(lat)
    a = vmc.eval_config(T, lat, spins)
    b = vmc.eval_config(transpose_tensors(T, lat), transposed(lat), transpose_spins(spins, lat))
    ratios = a["ratios"].copy()
    nh = lat.Ly * (lat.Lx - 1)
    for y in range(lat.Ly - 1):
        for x in range(lat.Lx):
            # the vertical bond (y,x)-(y+1,x) is horizontal bond (x,y)-(x,y+1) of the transposed lattice
            ratios[nh + y * lat.Lx + x] = b["ratios"][x * (lat.Ly - 1) + y]
    index = {(p, q): i for i, (p, q, _) in enumerate(bonds(lat))}
    e_loc = local_energy(lat, spins, lambda p, q: ratios[index[(p, q)]])
    return dict(sign=a["sign"], log_abs_psi=a["log_abs_psi"], e_loc=e_loc, dlnpsi=a["dlnpsi"], ratios=ratios)


def run_chain(T, lat, ch, n_burn, n_meas):
    """n_burn + n_meas sweeps (horizontal bonds by rows, then vertical bonds by columns);
    returns per measured sweep dict(sign, log_abs_psi, e_loc, dlnpsi, spins)."""
    _check(lat)
    lt, Tt = transposed(lat), transpose_tensors(T, lat)
    out = []
    for i in range(n_burn + n_meas):
        Dl = vmc._lower_boundaries(T, lat, ch.spins)
        vmc._top_down_pass(T, lat, ch, Dl, vertical=False)
        cht = vmc.Chain(lt, transpose_spins(ch.spins, lat), ch.seed, ch.lattice_id + COLUMN_KEY, ch.chain_id,
                        ch.sweep)
        vmc._top_down_pass(Tt, lt, cht, vmc._lower_boundaries(Tt, lt, cht.spins), vertical=False)
        ch.spins = untranspose_spins(cht.spins, lat)
        ch.accepted += cht.accepted
        ch.proposed += cht.proposed
        if i >= n_burn:
            o = eval_config(T, lat, ch.spins)
            out.append(dict(sign=o["sign"], log_abs_psi=o["log_abs_psi"], e_loc=o["e_loc"], dlnpsi=o["dlnpsi"],
                            spins=ch.spins.copy()))
        ch.sweep += 1
    return out
