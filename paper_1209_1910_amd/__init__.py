"""MI355X (gfx950) inverse iteration with compact-WY re-orthogonalization.

The compute path lives in the HIP C-ABI library ``libtridiag_eigvecs.so``
(sources under ``csrc/``); ``binding`` marshals arguments to it.  Importing the
package loads nothing: the library is opened on first use.
"""
