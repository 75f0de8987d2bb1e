"""Experiment drivers (run on an MI355X): each prints progress lines and one
JSON result line.  They use only the library's C ABI through the binding and
seeded synthetic inputs."""
