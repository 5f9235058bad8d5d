// Vector dimensions for which kernels are compiled.  One object file per
// entry is built from esg_search_inst.hip with -DESG_DIM=<d>.  A kernel
// depends on the dimension only through its lane shape (lanes per vector
// and chunks per lane for each storage type) and its padded row length, so
// the kernels compiled for one entry serve every dimension with the same
// shape and a row no longer than the entry's: the loader picks the first
// such entry (e.g. 128 serves 97..128).
#pragma once
#ifdef ESG_DIMS_ONLY   // a development build with the kernels of one class
#define ESG_DIMS_APPLY(X, d) X(d)
#define ESG_DIMS(X) ESG_DIMS_APPLY(X, ESG_DIMS_ONLY)
#else
#define ESG_DIMS(X) X(32) X(64) X(96) X(128) X(256) X(512) X(768) X(1024) X(2048)
#endif
