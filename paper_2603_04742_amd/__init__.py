"""Encrypted sparse matrix-vector multiplication over the CSSC format (arXiv 2603.04742) for
MI355X.  ``hespmv`` is the binding of the HIP library; ``workloads`` draws seeded synthetic inputs."""
