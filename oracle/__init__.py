"""CPU oracle for the nearest-neighbour conditional-mutual-information path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The product path (the HIP library and its Python binding) never
imports it, and this package imports nothing from the product.

The oracle is a plain, slow, deliberately unblocked-where-possible restatement
of what the path computes:

* ``harmonic``  - harmonic numbers H_n = sum_{m<=n} 1/m (the digamma values the
  estimator needs, since psi(n+1) = -gamma + H_n).
* ``ksg``       - the Kraskov-Stoegbauer-Grassberger nearest-neighbour estimator
  (algorithm 1 of Kraskov et al. 2004, the estimator the paper names in its
  Summary, estimator paragraph) in the conditional form of Frenzel & Pompe
  2007: max-norm k-th neighbour distance in the joint space, strict range
  counts in the XZ, YZ and Z subspaces, digamma sum.  A NumPy form (O1), a
  pure-Python loop form (O2) and an exact rational form.
* ``stats``     - lagged embedding of candidate past variables, the surrogate
  max-statistic test, greedy parent selection gated by that test and the
  omnibus test (Summary, network-inference paragraph: greedy maximisation of
  a CMI criterion, gated by surrogate null distributions).
* ``features`` / ``mlp`` - the learned-null gate's feature vector and the
  16-64-64-2 multilayer perceptron (forward, backward, Adam) in FP64.

Readings of the paper used here (it gives no formulas) are listed in each
function's docstring.
"""
