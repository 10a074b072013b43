"""MI355X-native FGraft harvest (arxiv 2609.30493): HIP kernels behind a
C-ABI (include/fgraft.h); ``fgraft`` is the Python binding, ``datagen`` the
seeded synthetic inputs.  Importing the package loads nothing: the library is
loaded on the first call and its absence raises."""
