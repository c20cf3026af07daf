"""MI355X-native exact pair counting (FCFC hot path) -- Python binding package.

The compute path lives in the HIP library ``csrc`` builds (libfcfc.so); this
package only marshals arguments to its C ABI (see ``fcfc.py``).
"""
__all__ = ["synth"]
