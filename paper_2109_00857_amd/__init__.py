"""MI355X-native stochastic-flow MDP planner.

Builds the sparse MDP of a marine-vehicle path-planning problem (transition
counts and expected one-step rewards from a reduced-order stochastic flow),
solves it by value iteration and extracts the greedy policy, with hand-written
HIP kernels for gfx950 behind a C ABI (``include/mdp.h``).
"""
