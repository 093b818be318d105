"""Plain FP64 CPU oracle of the TNMCMC-1 slice proposal (arXiv 2509.23945).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, to check and to time against.

It is written from the paper, slowly and plainly, with numpy's QR and SVD as
library steps and no blocking or fusion beyond what the method states:

* ``philox``  - the counter-based generator both sides draw their uniforms from
* ``model``   - energies, the held layers' field on a slice, observables
* ``bmps``    - boundary-MPS environments with QR + truncated SVD to chi
* ``sampler`` - ancestral sampling with exact log q, and teacher forcing
* ``chain``   - Metropolis-Hastings slice update and even/odd sweeps
* ``autocorr``- integrated autocorrelation time
* ``nn``      - the learned autoregressive proposal: masked-convolution
  network, log q, sampling, loss gradient, Adam and its MH slice update

Every part is pinned by the ``-m "not gpu"`` tests against brute-force
enumeration, row transfer matrices, closed forms, exact stationarity and a
library generator; none is "parity unpinned".
"""
from . import autocorr, bmps, chain, model, nn, philox, sampler  # noqa: F401
