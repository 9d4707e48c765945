"""ctypes binding of libs7.so (filled in with the library)."""
