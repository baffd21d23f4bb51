"""FP64 CPU oracle for the PTSBE hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  It
shares no code with the GPU library (``paper_2604_08467_amd``) and never imports
it; the only module both sides use is ``workloads`` (seeded input generators).

It computes, plainly and slowly, what the method computes (Sec. II-B, III-A,
III-B of the paper):

* ``philox``       - Philox4x32-10 counter-based generator (Salmon et al., SC'11)
* ``upv``          - noise proposal probabilities and the unified-path-variation
                     merge of a gate with its sampled Kraus operators (Sec. III-A)
* ``pts``          - pre-trajectory sampling of unique error sets (Sec. II-C)
* ``statevector``  - dense FP64 statevector of a trajectory, explicit-insertion
                     variant, textbook density-matrix diagonal (pins)
* ``tn``           - explicit ket / doubled tensor networks for one batch with the
                     prefix projected, contracted pairwise with numpy einsum
* ``lightcone``    - the gates a doubled network keeps under the light cone
                     (forward reachability over the gate dependency graph)
* ``sampling``     - batch-wise conditional marginals and the per-shot sampler
                     (Sec. II-B), NBS bookkeeping (Sec. III-B), trajectory weights

Every function names the passage it follows and is pinned by the CPU tests of
the oracle against closed forms, invariants or brute force; the Philox
generator's cross-implementation parity is unpinned (no published known-answer
vectors are available here).
"""
