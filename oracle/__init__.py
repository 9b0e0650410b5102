"""CPU oracle for batched recursive Green's function (RGF) selected inversion.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link anything in this package: only the tests, the smoke entry point and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path.

Everything here is plain, slow and meant to be checked by eye against the
paper (arXiv 2508.19138, "QuaTrEx"):

* ``rgf``      - the forward/backward block recursions of Sec. 3.2.3
                 (Eqs. forward-pass and backward-pass), general form.
* ``dense``    - the plain definition of the result: X^R = A^{-1} and
                 X^s = A^{-1} B^s A^{-dagger} (Eq. system-solve), selected blocks.
* ``assembly`` - the system matrices of Table "quantities" / Sec. 3.2.2:
                 G-type  A = E S - H - Sigma^R,  B^s = Sigma^s;
                 W-type  A = I - trunc(V P^R),   B^s = trunc(V P^s V^dagger).
* ``chain``    - closed-form Green's function of a uniform 1-D tight-binding
                 chain with exact lead self-energies (independent pin).
* ``tridiag``  - closed-form inverse of a scalar tridiagonal matrix via
                 continuants (independent pin for block size 1).
* ``observables`` - local density of states, charge density and current
                 from the selected blocks (Sec. "Observables").
* ``convolution`` - the element-wise energy convolution of two descriptors
                 that forms the scattering terms (Sec. "Energy
                 Convolutions", Eq. interaction).
* ``nested``   - nested-dissection selected inversion (the partitioned
                 solver of Sec. 4.4): per-partition elimination, the reduced
                 system on the separators, per-partition recovery.
* ``obc``      - the lead surface function of Sec. "Retarded OBC": the
                 fixed-point iteration of Eq. (naive) and Sancho-Rubio
                 decimation, the boundary block n x n', and the
                 lesser/greater blocks by fluctuation-dissipation.
* ``flops``    - the canonical flop model used to price a solve.

All arithmetic is complex128 (IEEE binary64), the paper's precision.
"""

from .rgf import rgf_selected
from .dense import dense_from_bt, dense_selected
from .assembly import assemble_g, assemble_w, w_retarded_diag
from .chain import chain_closed_form, chain_lead_self_energy
from .tridiag import tridiag_inverse_selected
from .flops import rgf_flops, w_assembly_flops
from .obc import (obc_fixed_point, obc_sancho_rubio, obc_sancho_rubio_steps,
                  obc_lesser_greater, obc_lyapunov_fixed_point, obc_lyapunov_doubling)
from .observables import observables
from .convolution import energy_convolution

__all__ = [
    "rgf_selected", "dense_from_bt", "dense_selected",
    "assemble_g", "assemble_w", "w_retarded_diag", "chain_closed_form",
    "chain_lead_self_energy", "tridiag_inverse_selected", "rgf_flops",
    "w_assembly_flops", "obc_fixed_point", "obc_sancho_rubio",
    "obc_sancho_rubio_steps", "obc_lesser_greater", "observables",
    "obc_lyapunov_fixed_point", "obc_lyapunov_doubling", "energy_convolution",
]
