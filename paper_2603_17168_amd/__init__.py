"""MI355X-native cache-semantic GPU hash table (arxiv 2603.17168, "HierarchicalKV").

``cskv.Table`` binds the HIP library built from ``csrc/``; ``workload`` holds the seeded input
generators.  Importing the package loads nothing; the library is loaded on first use.
"""
