"""q2sv: UCCSD state-vector simulation on one MI355X (gfx950).

* ``binding``  -- ctypes binding of libq2sv.so with the C names
* ``problem``  -- JW Pauli-sum Hamiltonian and UCCSD rotation list builders
* ``engine``   -- device-resident states, Hamiltonians and the UCC energy
                  ``torch.autograd.Function``
* ``serve``    -- continuous-batching request loop
* ``build``    -- hipcc build of the library
"""
