"""CPU oracle of the FIZI/Mouse pipeline. Test infrastructure only."""
